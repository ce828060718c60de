// Batched apply: y_r = sgn(H_w(mu)) x_r for several sources of one field, the
// Schur-deflated modified Arnoldi of Section 5.2 run on every x_r with the
// shared partial Schur pair (S_m, T_m) and links.
//
// The active right-hand sides advance in lockstep: per Arnoldi step one
// stencil launch, one dot pass and one update pass carry every active slot
// (the slot map travels in the kernel arguments).  At a checkpoint the
// small-matrix signs of all active slots run as one batch, each matrix
// stopping on its own test; a slot whose coefficient change fell below tol
// (or whose Krylov space became invariant) is assembled, y_r = Q_r c_r
// (Eq. eq:formula), and leaves the active set.  Per slot the arithmetic is
// that of sgn_apply (same kernels, same reduction order, same source
// projection), so at a fixed Krylov dimension the result is bitwise the
// single-source result.  With a tolerance the batch shares its checkpoints,
// placed for its slowest member, so a slot can stop at a later even k than
// it would alone.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <map>
#include <vector>

#include "ckpt.h"
#include "context.h"

namespace {

int even_k(int k) { return (k + 1) & ~1; }

// (re)allocate the batch workspace for nslots sources and kcap Krylov vectors
void batch_ensure(sgn_ctx* c, int nslots, int kcap) {
  BatchWork& b = c->bw;
  const bool same_layout = b.V && b.prec == c->prec && b.m == c->m && b.lrm == c->lr_m;
  if (same_layout && b.nslots >= nslots && b.kcap >= kcap) return;
  if (same_layout) {
    nslots = std::max(nslots, b.nslots);
    kcap = std::max(kcap, b.kcap);
  }
  b.release();
  const int m = c->m;
  const size_t ldq = c->ldq, S = (size_t)nslots;
  b.nslots = nslots;
  b.kcap = kcap;
  b.m = m;
  b.lrm = c->lr_m;
  b.prec = c->prec;
  b.ldq = ldq;
  b.ncap = m + kcap + 1;
  const size_t vt = b.vt(), ncap = (size_t)b.ncap, n = (size_t)m + kcap, mm = (size_t)std::max(m, 1);
  b.vstride = ldq * (size_t)(kcap + 1);
  SGN_HIP(hipMalloc(&b.V, vt * b.vstride * S));
  SGN_HIP(hipMalloc(&b.u, sizeof(double2) * ldq * 2 * S));
  if (b.prec == SGN_PREC_MIXED) SGN_HIP(hipMalloc(&b.ulo, vt * ldq * 2 * S));
  SGN_HIP(hipMalloc(&b.z, vt * ldq * S));
  SGN_HIP(hipMalloc(&b.xin, sizeof(double2) * ldq * S));
  SGN_HIP(hipMalloc(&b.y, sizeof(double2) * ldq * S));
  SGN_HIP(hipMalloc(&b.H, sizeof(double2) * ncap * ncap * S));
  // two n x n blocks per slot: the patched composite matrix and its sign
  SGN_HIP(hipMalloc(&b.F, sizeof(double2) * n * n * 2 * S));
  SGN_HIP(hipMalloc(&b.c0, sizeof(double2) * mm * S));
  SGN_HIP(hipMalloc(&b.lrc, sizeof(double2) * (size_t)std::max(c->lr_m, 1) * S));
  SGN_HIP(hipMalloc(&b.cv, sizeof(double2) * ncap * 2 * S));
  for (double** p : {&b.beta, &b.err, &b.ref, &b.inv}) SGN_HIP(hipMalloc(p, sizeof(double) * S));
  for (int** p : {&b.flag, &b.fin}) SGN_HIP(hipMalloc(p, sizeof(int) * S));
  SGN_HIP(hipHostMalloc(&b.hpin, sizeof(double) * 4 * S, hipHostMallocDefault));
  SGN_HIP(hipMalloc(&b.jdev, sizeof(int)));
  gs_alloc(b.gs, c->N, ldq, std::max((int)mm, c->lr_m));
  krylov_alloc(b.kw, c->N, ldq, b.ncap, nslots);
  dense_reserve(b.dense, (int)n, nslots);
  // the Schur block T_m of every slot's composite matrix never changes
  SGN_HIP(hipMemset(b.H, 0, sizeof(double2) * ncap * ncap * S));
  for (int r = 0; r < nslots && m > 0; ++r) dev_copy_mat(c->Tdev, m, b.H + (size_t)r * ncap * ncap, b.ncap, m, m, nullptr);
  SGN_HIP(hipDeviceSynchronize());
}

struct SlotResult {
  int k = 0;
  bool done = false, converged = false, breakdown = false;
  double err = 1e30;
};

// one chunk of at most kMaxBatch sources; fixed_k >= 0: exactly that many steps
int run_batch(sgn_ctx* c, int nr, const double2* X_abi, double2* Y_abi, double tol, int kmax, int fixed_k,
              sgn_info* info) {
  const auto t_start = std::chrono::steady_clock::now();
  hipStream_t s = c->stream;
  Profiler* prof = c->prof.on ? &c->prof : nullptr;
  c->prof.stream = s;
  const int m = c->m, N = c->N;
  const size_t ldq = c->ldq;
  const int kwant = fixed_k >= 0 ? fixed_k : kmax;
  batch_ensure(c, nr, std::max(kwant, 2));
  BatchWork& b = c->bw;
  const bool mixed = (b.prec == SGN_PREC_MIXED);
  const size_t ns = (size_t)b.nslots, ncap = (size_t)b.ncap, mm = (size_t)std::max(m, 1);
  double* h_err = b.hpin;
  double* h_beta = b.hpin + ns;
  int* h_flag = reinterpret_cast<int*>(b.hpin + 2 * ns);
  int* h_fin = h_flag + ns;

  // step (iii) per source, as in sgn_apply: one Gram-Schmidt pass against S
  // now, its re-orthogonalisation folded into Arnoldi step 0
  SGN_HIP(hipMemsetAsync(b.flag, 0, sizeof(int) * ns, s));
  SGN_HIP(hipMemsetAsync(b.fin, 0, sizeof(int) * ns, s));
  for (int r = 0; r < nr; ++r) {
    double2* xr = b.xin + (size_t)r * ldq;
    double2* u0 = b.u + (size_t)r * ldq;
    wilson_pack(c->lat, X_abi + (size_t)r * N, xr, s);
    dev_check_finite(xr, (size_t)N, b.fin + r, s);
    SGN_HIP(hipMemcpyAsync(u0, xr, sizeof(double2) * N, hipMemcpyDeviceToDevice, s));
    gs_norm(b.gs, N, xr, b.ref + r, b.inv + r, nullptr, s, prof);
    SGN_HIP(hipMemcpyAsync(b.kw.sc + (size_t)r * kScStride + kScRef, b.ref + r, sizeof(double),
                           hipMemcpyDeviceToDevice, s));
    if (m > 0) {
      gs_dot(b.gs, c->S, ldq, N, m, u0, b.c0 + (size_t)r * mm, s, prof);
      gs_update(b.gs, c->S, ldq, N, m, b.c0 + (size_t)r * mm, u0, nullptr, 0, s, prof);
    }
    if (c->lr_m > 0) {  // LR-deflation, step (iii): L^dag x, x_- = (1 - R L^dag) x
      double2* lc = b.lrc + (size_t)r * c->lr_m;
      gs_dot(b.gs, c->lrL, ldq, N, c->lr_m, u0, lc, s, prof);
      gs_update(b.gs, c->lrR, ldq, N, c->lr_m, lc, u0, nullptr, 0, s, prof);
    }
    if (mixed) dev_to_f32(u0, static_cast<float2*>(b.ulo) + (size_t)r * ldq, (size_t)N, s);
  }
  SGN_HIP(hipMemcpyAsync(h_fin, b.fin, sizeof(int) * nr, hipMemcpyDeviceToHost, s));
  SGN_HIP(hipStreamSynchronize(s));
  for (int r = 0; r < nr; ++r)
    if (h_fin[r] != 0) throw SgnError{SGN_EINVAL, "x contains NaN or Inf"};

  KrylovArgs base;
  base.tune = c->tune;
  base.N = N;
  base.ldq = ldq;
  base.m = m;
  base.S = c->S;
  base.V = b.V;
  base.vstride = b.vstride;
  base.ustride = ldq;
  base.z = b.z;
  base.zstride = ldq;
  base.H = b.H;
  base.ldh = b.ncap;
  base.hstride = ncap * ncap;
  base.c0 = b.c0;
  base.c0stride = (int)mm;
  base.beta = b.beta;
  base.flag = b.flag;
  base.brk_tol = mixed ? 1e-6 : 1e-12;
  auto half_u = [&](int p) { return b.u + (size_t)(p & 1) * ns * ldq; };
  auto half_lo = [&](int p) { return static_cast<float2*>(b.ulo) + (size_t)(p & 1) * ns * ldq; };
  auto fill = [&](KrylovArgs& ka, const std::vector<int>& slots, int j) {
    ka.nb = (int)slots.size();
    for (int z = 0; z < ka.nb; ++z) {
      ka.act[z] = slots[z];
      ka.jv[z] = j;
    }
  };

  std::vector<SlotResult> res(nr);
  std::vector<int> nprev(nr, -1);
  std::vector<int> active(nr);
  for (int r = 0; r < nr; ++r) active[r] = r;
  int ncheck = 0, newton_total = 0, n_matvec = 0;
  double ms_sign = 0.0;
  CkModel model;  // largest change among the running slots, per span
  int prev_ck = -1;
  int next_ck;
  const bool hinted = b.k_hint > 0 && b.tol_hint == tol;
  if (fixed_k >= 0)
    next_ck = fixed_k;
  else if (hinted)
    next_ck = std::min(kmax, std::max(2, even_k(b.k_hint)));
  else
    next_ck = std::min(kmax, std::max(2, even_k(std::min(32, kmax / 2))));

  // assemble y_r = Q_r c_r for finished slots (grouped by their dimension)
  auto finish = [&](const std::vector<int>& slots, const double2* cvcur) {
    std::map<int, std::vector<int>> byn;
    for (int r : slots) byn[m + res[r].k].push_back(r);
    for (auto& g : byn) {
      KrylovArgs kf = base;
      fill(kf, g.second, 0);
      if (mixed)
        krylov_combine<float2>(b.kw, kf, cvcur, (int)ncap, b.y, ldq, g.first, s, prof);
      else
        krylov_combine<double2>(b.kw, kf, cvcur, (int)ncap, b.y, ldq, g.first, s, prof);
      for (int r : g.second) {
        if (c->lr_m > 0) {  // LR-deflation, step (vi): y += R sgn(Lambda) L^dag x
          double2* lc = b.lrc + (size_t)r * c->lr_m;
          dev_cmul(c->lrSgn, lc, c->lr_m, s);
          gs_add(b.gs, c->lrR, ldq, N, c->lr_m, lc, b.y + (size_t)r * ldq, s, prof);
        }
        wilson_unpack(c->lat, b.y + (size_t)r * ldq, Y_abi + (size_t)r * N, s);
      }
    }
  };

  // checkpoint (step (v)) for every active slot after k steps; returns false
  // once no slot is left
  auto checkpoint = [&](int k) -> bool {
    const auto t0 = std::chrono::steady_clock::now();
    SGN_HIP(hipMemcpyAsync(h_flag, b.flag, sizeof(int) * nr, hipMemcpyDeviceToHost, s));
    SGN_HIP(hipStreamSynchronize(s));
    std::map<int, std::vector<int>> groups;  // Krylov dimension -> slots
    for (int r : active) {
      const int f = h_flag[r];
      if (f < 0) throw SgnError{SGN_EINVAL, "non-finite value in the Krylov basis"};
      res[r].breakdown = f > 0;
      res[r].k = f > 0 ? f - 1 : k;
      groups[res[r].k].push_back(r);
    }
    double2* cvcur = b.cv + (size_t)(ncheck & 1) * ns * ncap;
    double2* cvprev = b.cv + (size_t)((ncheck + 1) & 1) * ns * ncap;
    for (auto& g : groups) {
      const int kk = g.first, n = m + kk, nb = (int)g.second.size();
      const size_t nn = (size_t)n * n;
      double2* Apat = b.F;
      double2* Fout = b.F + nn * ns;
      if (n > 0) {
        KrylovArgs kc = base;
        fill(kc, g.second, kk);
        kc.u = half_u(k);
        if (kk > 0) {
          // finish the re-orthogonalisation of the last column, on a copy
          if (mixed)
            krylov_dot<float2>(b.kw, kc, false, s, prof);
          else
            krylov_dot<double2>(b.kw, kc, false, s, prof);
        }
        krylov_patch(b.kw, kc, n, Apat, nn, kk > 0, s);
        const int it = dense_sign_batched(b.dense, n, nb, Apat, n, nn, Fout, n, nn, s, prof);
        newton_total += std::max(it, 0);
      }
      SlotMap cm;
      cm.n = nb;
      for (int z = 0; z < nb; ++z) {
        cm.slot[z] = g.second[z];
        cm.aux[z] = nprev[g.second[z]];
      }
      dense_coeffs_batched(n, m, Fout, n, nn, b.c0, (int)mm, b.beta, cvcur, cvprev, (int)ncap, cm, b.err, s);
    }
    SGN_HIP(hipMemcpyAsync(h_err, b.err, sizeof(double) * nr, hipMemcpyDeviceToHost, s));
    SGN_HIP(hipStreamSynchronize(s));
    ms_sign += std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    ++ncheck;
    std::vector<int> done_now, still;
    double worst = 0.0;
    // rate of the error model: the batch's spans so far (the worst change of
    // each) or the first batched apply on this field; this span's own change
    // per slot
    double rate = model.rate(b.rate_hint < 0.0 ? b.rate_hint : 0.0);
    if (prev_ck >= 0) {
      double w = 0.0;
      for (int r : active) w = std::max(w, h_err[r]);
      if (w < 1e29) {
        CkModel probe = model;
        probe.hist.push_back(CkSpan{prev_ck, k, w});
        rate = probe.rate(rate);
      }
    }
    for (int r : active) {
      const double e = h_err[r];
      res[r].err = e;
      nprev[r] = m + res[r].k;
      const bool ok = prev_ck >= 0 && e < 1e29 && CkModel::bound(e, k - prev_ck, rate) <= tol;
      if (fixed_k >= 0 || res[r].breakdown || ok || k == kwant) {
        res[r].done = true;
        res[r].converged = fixed_k >= 0 || res[r].breakdown || ok;
        done_now.push_back(r);
      } else {
        still.push_back(r);
        worst = std::max(worst, e);
      }
    }
    if (!done_now.empty()) finish(done_now, cvcur);
    if (still.empty() && fixed_k < 0 && b.k_hint == 0 && prev_ck > 0) {
      // remember where the batch was certified (checkpoint placement only)
      b.k_hint = prev_ck;
      b.tol_hint = tol;
    }
    active.swap(still);
    if (active.empty()) return false;
    // next checkpoint from the geometric error model of sgn_apply, on the
    // largest change among the slots still running
    if (prev_ck >= 0 && worst < 1e29) model.hist.push_back(CkSpan{prev_ck, k, worst});
    prev_ck = k;
    rate = model.rate(b.rate_hint < 0.0 ? b.rate_hint : 0.0);
    if (model.hist.size() >= 2 && CkModel::usable(rate) && b.rate_hint == 0.0) b.rate_hint = rate;
    next_ck = model.next(k, kwant, tol, rate, hinted && model.hist.empty());
    return true;
  };

  if (kwant == 0) {
    // no Krylov part: y = S sgn(T_m) S^dag x
    SGN_HIP(hipMemsetAsync(b.beta, 0, sizeof(double) * ns, s));
    checkpoint(0);
  }
  // one Arnoldi step for the running slots at step j (step (iv)); with
  // jdev set, the launch slots read the step index from the device
  auto step = [&](KrylovArgs ka, int j, hipStream_t st, Profiler* pf) {
    SlotMap map;
    map.n = ka.nb;
    for (int z = 0; z < map.n; ++z) map.slot[z] = ka.act[z];
    ka.u = half_u(j);
    ka.unext = half_u(j + 1);
    if (mixed) {
      wilson_apply_slots<float2>(c->lat, c->links32, half_lo(j), ldq, static_cast<float2*>(b.z), ldq, map, st, pf);
      ka.ulonext = half_lo(j + 1);
      krylov_dot<float2>(b.kw, ka, true, st, pf);
      krylov_update<float2>(b.kw, ka, st, pf);
    } else {
      wilson_apply_slots<double2>(c->lat, c->links, half_u(j), ldq, static_cast<double2*>(b.z), ldq, map, st, pf);
      ka.ulonext = nullptr;
      krylov_dot<double2>(b.kw, ka, true, st, pf);
      krylov_update<double2>(b.kw, ka, st, pf);
    }
  };
  // captured run of L steps (L even) from any even step j of the same
  // 32-column bucket, for the current set of running slots: the same kernels
  // and arguments as direct launches (the candidate halves alternate with the
  // step's parity, which an even start fixes), so results are bitwise the same
  auto graph_for = [&](int j, int L) -> hipGraphExec_t {
    const int bucket = (j + L - 1) / 32;
    auto key = std::make_pair(active, bucket);
    auto it = b.graphs.find(key);
    if (it != b.graphs.end()) return it->second;
    const int jcap = std::min(32 * (bucket + 1) - 1, b.kcap - 1);
    SGN_REQUIRE(j + L - 1 <= jcap, SGN_EINVAL, "captured steps exceed the workspace");
    if (!c->cap_stream) SGN_HIP(hipStreamCreateWithFlags(&c->cap_stream, hipStreamNonBlocking));
    hipStream_t cs = c->cap_stream;
    KrylovArgs ka = base;
    fill(ka, active, jcap);
    ka.jdev = b.jdev;
    hipGraph_t g = nullptr;
    SGN_HIP(hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal));
    try {
      for (int t = 0; t < L; ++t) {
        ka.joff = t;
        step(ka, t, cs, nullptr);
      }
      krylov_set_index(b.jdev, L, true, cs);
    } catch (...) {
      (void)hipStreamEndCapture(cs, &g);
      if (g) (void)hipGraphDestroy(g);
      throw;
    }
    SGN_HIP(hipStreamEndCapture(cs, &g));
    hipGraphExec_t ex = nullptr;
    const hipError_t e = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    SGN_HIP(e);
    b.graphs[key] = ex;
    return ex;
  };
  const int L = c->graph_steps & ~1;
  for (int j = 0; j < kwant && !active.empty();) {
    const int seg_end = std::min(next_ck, kwant);
    if (L > 0 && !prof && (j & 1) == 0 && j + L <= seg_end) {
      // whole captured runs up to the checkpoint
      krylov_set_index(b.jdev, j, false, s);
      while (j + L <= seg_end) {
        SGN_HIP(hipGraphLaunch(graph_for(j, L), s));
        j += L;
        n_matvec += L * (int)active.size();
      }
      if (j == next_ck || j == kwant)
        if (!checkpoint(j)) break;
      continue;
    }
    KrylovArgs ka = base;
    fill(ka, active, j);
    step(ka, j, s, prof);
    const int k = ++j;
    n_matvec += (int)active.size();
    if (k == next_ck || k == kwant)
      if (!checkpoint(k)) break;
  }
  SGN_HIP(hipMemcpyAsync(h_beta, b.beta, sizeof(double) * nr, hipMemcpyDeviceToHost, s));
  SGN_HIP(hipStreamSynchronize(s));
  if (prof) c->prof.flush();
  const double ms_total =
      std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t_start).count();
  bool all = true;
  sgn_info agg{};
  for (int r = 0; r < nr; ++r) {
    sgn_info in{};
    in.k_used = res[r].k;
    in.converged = res[r].converged ? 1 : 0;
    in.newton_iters = newton_total;
    in.n_matvec = res[r].k;
    in.n_checkpoints = ncheck;
    in.breakdown = res[r].breakdown ? 1 : 0;
    in.err_est = res[r].err;
    in.beta = h_beta[r];
    in.ms_sign = ms_sign;
    in.ms_total = ms_total;
    in.ms_arnoldi = ms_total - ms_sign;
    if (info) info[r] = in;
    all = all && res[r].converged;
    agg.k_used = std::max(agg.k_used, in.k_used);
    agg.err_est = std::max(agg.err_est, in.err_est);
  }
  agg.converged = all ? 1 : 0;
  agg.newton_iters = newton_total;
  agg.n_matvec = n_matvec;
  agg.n_checkpoints = ncheck;
  agg.ms_sign = ms_sign;
  agg.ms_total = ms_total;
  agg.ms_arnoldi = ms_total - ms_sign;
  c->info = agg;
  if (!all) {
    c->last_error = "kmax reached before the requested tolerance";
    return SGN_ENOCONV;
  }
  return SGN_OK;
}

// The batch with the block (s-step) process (sgn_set_block_steps, FP64): per
// source the start of sgn_apply's block process (two Gram-Schmidt passes
// against S, v_1 = x_perp / beta), then blocks of s steps for every running
// slot per launch, with run_batch's shared checkpoints (on whole blocks) and
// stopping rule.  Per slot the arithmetic is that of sgn_apply with the same
// block size, so at a fixed Krylov dimension a slot's result is bitwise the
// single-source one.  A block that is not of full rank throws BlockFallback
// (the caller repeats the batch with one-vector steps).
int run_batch_block(sgn_ctx* c, int nr, const double2* X_abi, double2* Y_abi, double tol, int kmax, int fixed_k,
                    sgn_info* info) {
  const auto t_start = std::chrono::steady_clock::now();
  hipStream_t s = c->stream;
  Profiler* prof = c->prof.on ? &c->prof : nullptr;
  c->prof.stream = s;
  const int m = c->m, N = c->N, sblk = c->block_s;
  const size_t ldq = c->ldq;
  const int kwant = fixed_k >= 0 ? fixed_k : kmax;
  batch_ensure(c, nr, std::max(kwant, 2));
  BatchWork& b = c->bw;
  const size_t ns = (size_t)b.nslots, ncap = (size_t)b.ncap, mm = (size_t)std::max(m, 1);
  if (b.blk.ncap < b.ncap || b.blk.nslots < b.nslots) block_alloc(b.blk, N, ldq, b.ncap, b.nslots);
  if (!(c->cheb_e > 0.0)) c->cheb_e = std::sqrt(sq_radius_estimate(c, 40, 0x5eedull));
  double* h_err = b.hpin;
  double* h_beta = b.hpin + ns;
  int* h_flag = reinterpret_cast<int*>(b.hpin + 2 * ns);
  int* h_fin = h_flag + ns;
  auto align = [&](int kk) { return std::min(kwant, (kk + sblk - 1) / sblk * sblk); };

  // step (iii) per source: two passes against S, c0 = S^dag x, beta, 1/beta
  SGN_HIP(hipMemsetAsync(b.flag, 0, sizeof(int) * ns, s));
  SGN_HIP(hipMemsetAsync(b.fin, 0, sizeof(int) * ns, s));
  SGN_HIP(hipMemsetAsync(b.blk.flag, 0, sizeof(int) * ns, s));
  for (int r = 0; r < nr; ++r) {
    double2* xr = b.xin + (size_t)r * ldq;
    double2* u0 = b.u + (size_t)r * ldq;
    wilson_pack(c->lat, X_abi + (size_t)r * N, xr, s);
    dev_check_finite(xr, (size_t)N, b.fin + r, s);
    SGN_HIP(hipMemcpyAsync(u0, xr, sizeof(double2) * N, hipMemcpyDeviceToDevice, s));
    if (c->lr_m > 0) {  // LR-deflation, step (iii): L^dag x, x_- = (1 - R L^dag) x
      double2* lc = b.lrc + (size_t)r * c->lr_m;
      gs_dot(b.gs, c->lrL, ldq, N, c->lr_m, u0, lc, s, prof);
      gs_update(b.gs, c->lrR, ldq, N, c->lr_m, lc, u0, nullptr, 0, s, prof);
    }
    if (m > 0) {
      double2* hout = b.cv + (size_t)r * ncap;         // m sums, then beta
      double2* h1 = b.cv + (ns + (size_t)r) * ncap;    // first-pass coefficients
      double2* h2 = b.F + (size_t)r * mm;              // second-pass coefficients
      gs_dot(b.gs, c->S, ldq, N, m, u0, h1, s, prof);
      gs_update(b.gs, c->S, ldq, N, m, h1, u0, nullptr, 0, s, prof);
      gs_dot(b.gs, c->S, ldq, N, m, u0, h2, s, prof);
      GsFinal fin{h1, hout, b.beta + r, b.inv + r, b.flag + r};
      gs_update(b.gs, c->S, ldq, N, m, h2, u0, &fin, 0, s, prof);
      SGN_HIP(hipMemcpyAsync(b.c0 + (size_t)r * mm, hout, sizeof(double2) * m, hipMemcpyDeviceToDevice, s));
    } else {
      gs_norm(b.gs, N, u0, b.beta + r, b.inv + r, b.flag + r, s, prof);
    }
  }
  SGN_HIP(hipMemcpyAsync(h_fin, b.fin, sizeof(int) * nr, hipMemcpyDeviceToHost, s));
  SGN_HIP(hipMemcpyAsync(h_flag, b.flag, sizeof(int) * nr, hipMemcpyDeviceToHost, s));
  SGN_HIP(hipStreamSynchronize(s));
  for (int r = 0; r < nr; ++r)
    if (h_fin[r] != 0 || h_flag[r] < 0) throw SgnError{SGN_EINVAL, "x contains NaN or Inf"};

  KrylovArgs base;
  base.tune = c->tune;
  base.N = N;
  base.ldq = ldq;
  base.m = m;
  base.S = c->S;
  base.V = b.V;
  base.vstride = b.vstride;
  base.ustride = ldq;
  base.z = b.z;
  base.zstride = ldq;
  base.H = b.H;
  base.ldh = b.ncap;
  base.hstride = ncap * ncap;
  base.c0 = b.c0;
  base.c0stride = (int)mm;
  base.beta = b.beta;
  base.flag = b.flag;
  base.brk_tol = 1e-12;
  base.u = b.u;
  auto fill = [&](KrylovArgs& ka, const std::vector<int>& slots, int j) {
    ka.nb = (int)slots.size();
    for (int z = 0; z < ka.nb; ++z) {
      ka.act[z] = slots[z];
      ka.jv[z] = j;
    }
  };
  BlockSpan span;
  span.S = c->S;
  span.V = static_cast<double2*>(b.V);
  span.vstride = b.vstride;
  span.ldq = ldq;
  span.m = m;
  span.N = N;
  span.ncap = b.ncap;
  span.H = b.H;
  span.hstride = ncap * ncap;
  span.ldh = b.ncap;
  auto span_for = [&](const std::vector<int>& slots) {
    BlockSpan sp = span;
    sp.nb = (int)slots.size();
    for (int z = 0; z < sp.nb; ++z) sp.act[z] = slots[z];
    return sp;
  };

  std::vector<SlotResult> res(nr);
  std::vector<int> nprev(nr, -1);
  std::vector<int> active, at_zero;  // x_perp = 0: y = S sgn(T) S^dag x, no Krylov step
  for (int r = 0; r < nr; ++r) (h_flag[r] > 0 ? at_zero : active).push_back(r);
  int ncheck = 0, newton_total = 0, n_matvec = 0;
  double ms_sign = 0.0;
  CkModel model;
  int prev_ck = -1;
  int next_ck;
  const bool hinted = b.k_hint > 0 && b.tol_hint == tol;
  if (fixed_k >= 0)
    next_ck = fixed_k;
  else if (hinted)
    next_ck = align(std::min(kmax, std::max(2, even_k(b.k_hint))));
  else
    next_ck = align(std::min(kmax, std::max(2, even_k(std::min(32, kmax / 2)))));

  // y_r = Q_r c_r for finished slots (grouped by their dimension)
  auto finish = [&](const std::vector<int>& slots, const double2* cvcur) {
    std::map<int, std::vector<int>> byn;
    for (int r : slots) byn[m + res[r].k].push_back(r);
    for (auto& g : byn) {
      KrylovArgs kf = base;
      fill(kf, g.second, 0);
      krylov_combine<double2>(b.kw, kf, cvcur, (int)ncap, b.y, ldq, g.first, s, prof);
      for (int r : g.second) {
        if (c->lr_m > 0) {
          double2* lc = b.lrc + (size_t)r * c->lr_m;
          dev_cmul(c->lrSgn, lc, c->lr_m, s);
          gs_add(b.gs, c->lrR, ldq, N, c->lr_m, lc, b.y + (size_t)r * ldq, s, prof);
        }
        wilson_unpack(c->lat, b.y + (size_t)r * ldq, Y_abi + (size_t)r * N, s);
      }
    }
  };

  // checkpoint (step (v)) for the slots of `slots` after k steps: signs,
  // coefficients, changes; the finished ones are assembled and leave
  auto checkpoint = [&](std::vector<int>& slots, int k) {
    const auto t0 = std::chrono::steady_clock::now();
    if (k > 0) {
      SGN_HIP(hipMemcpyAsync(h_flag, b.blk.flag, sizeof(int) * nr, hipMemcpyDeviceToHost, s));
      SGN_HIP(hipStreamSynchronize(s));
      for (int r : slots)
        if (h_flag[r] != 0) throw BlockFallback{};
    }
    for (int r : slots) {
      res[r].k = k;
      res[r].breakdown = (k == 0);
    }
    double2* cvcur = b.cv + (size_t)(ncheck & 1) * ns * ncap;
    double2* cvprev = b.cv + (size_t)((ncheck + 1) & 1) * ns * ncap;
    {
      const int n = m + k, nb = (int)slots.size();
      const size_t nn = (size_t)n * n;
      double2* Apat = b.F;
      double2* Fout = b.F + nn * ns;
      if (n > 0) {
        KrylovArgs kc = base;
        fill(kc, slots, k);
        krylov_patch(b.kw, kc, n, Apat, nn, false, s);
        const int it = dense_sign_batched(b.dense, n, nb, Apat, n, nn, Fout, n, nn, s, prof, c->cheb_e);
        newton_total += std::max(it, 0);
      }
      SlotMap cm;
      cm.n = nb;
      for (int z = 0; z < nb; ++z) {
        cm.slot[z] = slots[z];
        cm.aux[z] = nprev[slots[z]];
      }
      if (k == 0)
        for (int z = 0; z < nb; ++z) SGN_HIP(hipMemsetAsync(b.beta + slots[z], 0, sizeof(double), s));
      dense_coeffs_batched(n, m, Fout, n, nn, b.c0, (int)mm, b.beta, cvcur, cvprev, (int)ncap, cm, b.err, s);
    }
    SGN_HIP(hipMemcpyAsync(h_err, b.err, sizeof(double) * nr, hipMemcpyDeviceToHost, s));
    SGN_HIP(hipStreamSynchronize(s));
    ms_sign += std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    ++ncheck;
    std::vector<int> done_now, still;
    double worst = 0.0;
    double rate = model.rate(b.rate_hint < 0.0 ? b.rate_hint : 0.0);
    if (prev_ck >= 0) {
      double w = 0.0;
      for (int r : slots) w = std::max(w, h_err[r]);
      if (w < 1e29) {
        CkModel probe = model;
        probe.hist.push_back(CkSpan{prev_ck, k, w});
        rate = probe.rate(rate);
      }
    }
    for (int r : slots) {
      const double e = h_err[r];
      res[r].err = e;
      nprev[r] = m + res[r].k;
      const bool ok = prev_ck >= 0 && e < 1e29 && CkModel::bound(e, k - prev_ck, rate) <= tol;
      if (fixed_k >= 0 || res[r].breakdown || ok || k == kwant) {
        res[r].done = true;
        res[r].converged = fixed_k >= 0 || res[r].breakdown || ok;
        done_now.push_back(r);
      } else {
        still.push_back(r);
        worst = std::max(worst, e);
      }
    }
    if (!done_now.empty()) finish(done_now, cvcur);
    if (k == 0) {
      slots.swap(still);
      return;
    }
    if (still.empty() && fixed_k < 0 && b.k_hint == 0 && prev_ck > 0) {
      b.k_hint = prev_ck;
      b.tol_hint = tol;
    }
    slots.swap(still);
    if (slots.empty()) return;
    if (prev_ck >= 0 && worst < 1e29) model.hist.push_back(CkSpan{prev_ck, k, worst});
    prev_ck = k;
    rate = model.rate(b.rate_hint < 0.0 ? b.rate_hint : 0.0);
    if (model.hist.size() >= 2 && CkModel::usable(rate) && b.rate_hint == 0.0) b.rate_hint = rate;
    next_ck = align(model.next(k, kwant, tol, rate, hinted && model.hist.empty()));
  };

  if (!at_zero.empty()) checkpoint(at_zero, 0);
  if (kwant == 0 && !active.empty()) {
    // no Krylov part: y = S sgn(T_m) S^dag x
    checkpoint(active, 0);
  }
  if (!active.empty()) block_first(span_for(active), b.u, ldq, b.inv, 1, s);
  for (int j = 0; j < kwant && !active.empty();) {
    const int seg_end = std::min(next_ck, kwant);
    const int sb = std::min(sblk, seg_end - j);
    block_step(span_for(active), b.blk, c->lat, c->links, j, sb, c->cheb_e, s, prof);
    j += sb;
    n_matvec += sb * (int)active.size();
    if (j == next_ck || j == kwant) checkpoint(active, j);
  }
  SGN_HIP(hipMemcpyAsync(h_beta, b.beta, sizeof(double) * nr, hipMemcpyDeviceToHost, s));
  SGN_HIP(hipStreamSynchronize(s));
  if (prof) c->prof.flush();
  const double ms_total =
      std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t_start).count();
  bool all = true;
  sgn_info agg{};
  for (int r = 0; r < nr; ++r) {
    sgn_info in{};
    in.k_used = res[r].k;
    in.converged = res[r].converged ? 1 : 0;
    in.newton_iters = newton_total;
    in.n_matvec = res[r].k;
    in.n_checkpoints = ncheck;
    in.breakdown = res[r].breakdown ? 1 : 0;
    in.err_est = res[r].err;
    in.beta = h_beta[r];
    in.ms_sign = ms_sign;
    in.ms_total = ms_total;
    in.ms_arnoldi = ms_total - ms_sign;
    if (info) info[r] = in;
    all = all && res[r].converged;
    agg.k_used = std::max(agg.k_used, in.k_used);
    agg.err_est = std::max(agg.err_est, in.err_est);
  }
  agg.converged = all ? 1 : 0;
  agg.newton_iters = newton_total;
  agg.n_matvec = n_matvec;
  agg.n_checkpoints = ncheck;
  agg.ms_sign = ms_sign;
  agg.ms_total = ms_total;
  agg.ms_arnoldi = ms_total - ms_sign;
  c->info = agg;
  if (!all) {
    c->last_error = "kmax reached before the requested tolerance";
    return SGN_ENOCONV;
  }
  return SGN_OK;
}

int batched_entry(sgn_ctx* c, int nrhs, const double* X, double* Y, double tol, int kmax, int fixed_k,
                  sgn_info* info) {
  SGN_REQUIRE(nrhs >= 1, SGN_EINVAL, "nrhs must be positive");
  SGN_REQUIRE(X && Y, SGN_EINVAL, "X and Y must not be NULL");
  const double2* Xc = reinterpret_cast<const double2*>(X);
  double2* Yc = reinterpret_cast<double2*>(Y);
  int status = SGN_OK;
  for (int r0 = 0; r0 < nrhs; r0 += kMaxBatch) {
    const int nr = std::min(kMaxBatch, nrhs - r0);
    const double2* Xr = Xc + (size_t)r0 * c->N;
    double2* Yr = Yc + (size_t)r0 * c->N;
    sgn_info* ir = info ? info + r0 : nullptr;
    int st;
    if (c->block_s > 0 && c->prec == SGN_PREC_FP64) {
      try {
        st = run_batch_block(c, nr, Xr, Yr, tol, kmax, fixed_k, ir);
      } catch (const BlockFallback&) {
        st = run_batch(c, nr, Xr, Yr, tol, kmax, fixed_k, ir);
      }
    } else {
      st = run_batch(c, nr, Xr, Yr, tol, kmax, fixed_k, ir);
    }
    if (st != SGN_OK) status = st;
  }
  return status;
}

}  // namespace

extern "C" {

int sgn_apply_batched(sgn_ctx* c, int nrhs, const double* X, double* Y, double tol, int kmax, sgn_info* info) {
  return guarded(c, [&] {
    SGN_REQUIRE(tol > 0.0 && std::isfinite(tol), SGN_EINVAL, "tol must be positive");
    SGN_REQUIRE(kmax >= 2 && kmax <= c->N, SGN_EINVAL, "kmax must satisfy 2 <= kmax <= N");
    return batched_entry(c, nrhs, X, Y, tol, kmax, -1, info);
  });
}

int sgn_overlap_apply_batched(sgn_ctx* c, int nrhs, const double* X, double* Y, double tol, int kmax,
                              sgn_info* info) {
  return guarded(c, [&] {
    SGN_REQUIRE(tol > 0.0 && std::isfinite(tol), SGN_EINVAL, "tol must be positive");
    SGN_REQUIRE(kmax >= 2 && kmax <= c->N, SGN_EINVAL, "kmax must satisfy 2 <= kmax <= N");
    SGN_REQUIRE(X && Y && nrhs >= 1, SGN_EINVAL, "X and Y must not be NULL and nrhs >= 1");
    const size_t n = (size_t)nrhs * c->N;
    const auto px = reinterpret_cast<uintptr_t>(X), py = reinterpret_cast<uintptr_t>(Y);
    SGN_REQUIRE(px + n * sizeof(double2) <= py || py + n * sizeof(double2) <= px, SGN_EINVAL,
                "X and Y must not overlap");
    const int st = batched_entry(c, nrhs, X, Y, tol, kmax, -1, info);
    overlap_finish(reinterpret_cast<const double2*>(X), reinterpret_cast<double2*>(Y), n, c->stream);
    SGN_HIP(hipStreamSynchronize(c->stream));
    return st;
  });
}

int sgn_apply_batched_fixed(sgn_ctx* c, int nrhs, const double* X, double* Y, int k, sgn_info* info) {
  return guarded(c, [&] {
    SGN_REQUIRE(k >= 0 && k <= c->N - c->m - c->lr_m, SGN_EINVAL,
                "k must satisfy 0 <= k <= N - (deflation size)");
    return batched_entry(c, nrhs, X, Y, 1.0, std::max(k, 2), k, info);
  });
}

int sgn_apply_adjoint_batched(sgn_ctx* c, int nrhs, const double* X, double* Y, double tol, int kmax,
                              sgn_info* info) {
  return guarded(c, [&] {
    SGN_REQUIRE(tol > 0.0 && std::isfinite(tol), SGN_EINVAL, "tol must be positive");
    SGN_REQUIRE(kmax >= 2 && kmax <= c->N, SGN_EINVAL, "kmax must satisfy 2 <= kmax <= N");
    check_adjoint(c);
    AdjointScope scope(c);
    return batched_entry(c, nrhs, X, Y, tol, kmax, -1, info);
  });
}

int sgn_apply_adjoint_batched_fixed(sgn_ctx* c, int nrhs, const double* X, double* Y, int k, sgn_info* info) {
  return guarded(c, [&] {
    SGN_REQUIRE(k >= 0 && k <= c->N - c->m - c->lr_m, SGN_EINVAL,
                "k must satisfy 0 <= k <= N - (deflation size)");
    check_adjoint(c);
    AdjointScope scope(c);
    return batched_entry(c, nrhs, X, Y, 1.0, std::max(k, 2), k, info);
  });
}

}  // extern "C"
