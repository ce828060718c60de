// Serving session: continuous batching of y = sgn(H_w(mu)) x requests on one
// resident field (links, Schur pair and sgn(T_m) stay on the device).
//
// A session owns max_slots request slots, each with its own Krylov workspace
// (kmax vectors).  A request is admitted into a free slot when it is
// submitted (source projection, step (iii)); every session step then runs one
// Arnoldi step (step (iv)) for all occupied slots in one stencil, one dot and
// one update launch, each slot at its own Krylov dimension (the slot map and
// per-slot step index travel in the kernel arguments).  A slot reaching its
// own checkpoint evaluates the small composite sign (step (v)); when its
// coefficient change is <= its tol (or its space became invariant, or it hit
// its kmax) y = Q c is written to the caller's buffer (step (vi)) and the
// slot is free for the next request.
//
// A request's arithmetic depends only on the request: the kernels compute
// each slot exactly as they would alone, the small signs stop per matrix,
// and the checkpoint schedule uses the request's own history only (no
// field-level hints).  So a result is bitwise the same whatever else is in
// flight, and the same as sgn_apply on a fresh context.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <map>
#include <memory>
#include <string>
#include <vector>

#include "ckpt.h"
#include "context.h"

namespace {

int even_up2(int k) { return (k + 1) & ~1; }

struct Slot {
  bool busy = false;
  int req = -1;
  int j = 0;          // Arnoldi steps done
  int kreq = 0;       // this request's kmax
  double tol = 0.0;
  double2* y = nullptr;  // caller's output (device, ABI layout)
  int next_ck = 0, prev_ck = -1, nprev = -1, ncheck = 0, newton = 0;
  CkModel model;  // this request's changes between checkpoints
  double err = 1e30;
  double ms_sign = 0.0;
  std::chrono::steady_clock::time_point t0;
};

struct Done {
  int status = SGN_OK;
  sgn_info info{};
};

}  // namespace

struct sgn_session {
  sgn_ctx* c = nullptr;
  int max_slots = 0, kmax = 0, m = 0, ncap = 0, prec = SGN_PREC_FP64;
  size_t ldq = 0, vstride = 0;
  // device workspace, per slot at fixed strides
  void* V = nullptr;        // ldq x (kmax + 1), FP64 or FP32
  double2* u = nullptr;     // ldq, candidate (updated in place)
  void* ulo = nullptr;      // ldq, FP32 copy of the candidate (mixed)
  void* z = nullptr;        // ldq, stencil result
  double2* xin = nullptr;   // ldq, packed source
  double2* y = nullptr;     // ldq, packed result
  double2* H = nullptr;     // ncap x ncap composite Hessenberg
  double2* F = nullptr;     // 2 x (m + kmax)^2: patched composite, its sign
  double2* c0 = nullptr;    // max(m, 1)
  double2* lrc = nullptr;   // max(lr_m, 1): L^dag x of the LR-deflation
  double2* cv = nullptr;    // ncap, coefficients of the last checkpoint
  double2* cp = nullptr;    // ncap, coefficients of the one before
  double *beta = nullptr, *err = nullptr, *ref = nullptr, *inv = nullptr;
  int *flag = nullptr, *fin = nullptr;
  double* hpin = nullptr;   // pinned: err, flag, fin, beta per slot
  GsWork gs;
  KrylovWork kw;
  DenseWork dense;
  std::vector<Slot> slots;
  std::map<int, Done> done;
  int next_req = 0;

  size_t vt() const { return prec == SGN_PREC_MIXED ? sizeof(float2) : sizeof(double2); }

  void alloc() {
    const size_t S = (size_t)max_slots, nc = (size_t)ncap, n = (size_t)m + kmax, mm = (size_t)std::max(m, 1);
    vstride = ldq * (size_t)(kmax + 1);
    SGN_HIP(hipMalloc(&V, vt() * vstride * S));
    SGN_HIP(hipMalloc(&u, sizeof(double2) * ldq * S));
    if (prec == SGN_PREC_MIXED) SGN_HIP(hipMalloc(&ulo, vt() * ldq * S));
    SGN_HIP(hipMalloc(&z, vt() * ldq * S));
    SGN_HIP(hipMalloc(&xin, sizeof(double2) * ldq * S));
    SGN_HIP(hipMalloc(&y, sizeof(double2) * ldq * S));
    SGN_HIP(hipMalloc(&H, sizeof(double2) * nc * nc * S));
    SGN_HIP(hipMalloc(&F, sizeof(double2) * n * n * 2 * S));
    SGN_HIP(hipMalloc(&c0, sizeof(double2) * mm * S));
    SGN_HIP(hipMalloc(&lrc, sizeof(double2) * (size_t)std::max(c->lr_m, 1) * S));
    SGN_HIP(hipMalloc(&cv, sizeof(double2) * nc * S));
    SGN_HIP(hipMalloc(&cp, sizeof(double2) * nc * S));
    for (double** p : {&beta, &err, &ref, &inv}) SGN_HIP(hipMalloc(p, sizeof(double) * S));
    for (int** p : {&flag, &fin}) SGN_HIP(hipMalloc(p, sizeof(int) * S));
    SGN_HIP(hipHostMalloc(&hpin, sizeof(double) * 4 * S, hipHostMallocDefault));
    gs_alloc(gs, c->N, ldq, std::max((int)mm, c->lr_m));
    krylov_alloc(kw, c->N, ldq, ncap, max_slots);
    dense_reserve(dense, (int)n, max_slots);
    SGN_HIP(hipMemset(H, 0, sizeof(double2) * nc * nc * S));
    for (int r = 0; r < max_slots && m > 0; ++r) dev_copy_mat(c->Tdev, m, H + (size_t)r * nc * nc, ncap, m, m, nullptr);
    SGN_HIP(hipDeviceSynchronize());
  }

  void release() {
    (void)hipDeviceSynchronize();
    for (void** p : {&V, (void**)&u, &ulo, &z, (void**)&xin, (void**)&y, (void**)&H, (void**)&F, (void**)&c0,
                     (void**)&lrc, (void**)&cv, (void**)&cp, (void**)&beta, (void**)&err, (void**)&ref,
                     (void**)&inv, (void**)&flag, (void**)&fin})
      if (*p) {
        (void)hipFree(*p);
        *p = nullptr;
      }
    if (hpin) (void)hipHostFree(hpin);
    hpin = nullptr;
    gs_free(gs);
    krylov_free(kw);
    dense_destroy(dense);
  }

  KrylovArgs base() const {
    KrylovArgs a;
    a.tune = c->tune;
    a.N = c->N;
    a.ldq = ldq;
    a.m = m;
    a.S = c->S;
    a.V = V;
    a.vstride = vstride;
    a.u = u;
    a.unext = u;  // in place
    a.ustride = ldq;
    a.z = z;
    a.zstride = ldq;
    a.ulonext = prec == SGN_PREC_MIXED ? ulo : nullptr;
    a.H = H;
    a.ldh = ncap;
    a.hstride = (size_t)ncap * ncap;
    a.c0 = c0;
    a.c0stride = std::max(m, 1);
    a.beta = beta;
    a.flag = flag;
    a.brk_tol = prec == SGN_PREC_MIXED ? 1e-6 : 1e-12;
    return a;
  }

  // first checkpoint of a fresh request: as sgn_apply without a remembered k
  static int first_checkpoint(int kreq) { return std::min(kreq, std::max(2, even_up2(std::min(32, kreq / 2)))); }

  int submit(const double2* x_abi, double2* y_abi, double tol, int kreq) {
    SGN_REQUIRE(x_abi && y_abi, SGN_EINVAL, "x and y must not be NULL");
    SGN_REQUIRE(tol > 0.0 && std::isfinite(tol), SGN_EINVAL, "tol must be positive");
    SGN_REQUIRE(kreq >= 2 && kreq <= kmax, SGN_EINVAL, "kmax must satisfy 2 <= kmax <= the session's kmax");
    int r = -1;
    for (int q = 0; q < max_slots; ++q)
      if (!slots[q].busy) {
        r = q;
        break;
      }
    if (r < 0) return SGN_ENOMEM;
    hipStream_t s = c->stream;
    Profiler* prof = c->prof.on ? &c->prof : nullptr;
    c->prof.stream = s;
    const int N = c->N;
    const size_t mm = (size_t)std::max(m, 1);
    double2* xr = xin + (size_t)r * ldq;
    double2* ur = u + (size_t)r * ldq;
    // step (iii), as in sgn_apply: one Gram-Schmidt pass against S now, the
    // second folded into Arnoldi step 0
    SGN_HIP(hipMemsetAsync(flag + r, 0, sizeof(int), s));
    SGN_HIP(hipMemsetAsync(fin + r, 0, sizeof(int), s));
    wilson_pack(c->lat, x_abi, xr, s);
    dev_check_finite(xr, (size_t)N, fin + r, s);
    SGN_HIP(hipMemcpyAsync(ur, xr, sizeof(double2) * N, hipMemcpyDeviceToDevice, s));
    gs_norm(gs, N, xr, ref + r, inv + r, nullptr, s, prof);
    SGN_HIP(hipMemcpyAsync(kw.sc + (size_t)r * kScStride + kScRef, ref + r, sizeof(double), hipMemcpyDeviceToDevice,
                           s));
    if (m > 0) {
      gs_dot(gs, c->S, ldq, N, m, ur, c0 + (size_t)r * mm, s, prof);
      gs_update(gs, c->S, ldq, N, m, c0 + (size_t)r * mm, ur, nullptr, 0, s, prof);
    }
    if (c->lr_m > 0) {  // LR-deflation, step (iii): L^dag x, x_- = (1 - R L^dag) x
      double2* lc = lrc + (size_t)r * c->lr_m;
      gs_dot(gs, c->lrL, ldq, N, c->lr_m, ur, lc, s, prof);
      gs_update(gs, c->lrR, ldq, N, c->lr_m, lc, ur, nullptr, 0, s, prof);
    }
    if (prec == SGN_PREC_MIXED) dev_to_f32(ur, static_cast<float2*>(ulo) + (size_t)r * ldq, (size_t)N, s);
    int* h_fin = reinterpret_cast<int*>(hpin + max_slots) + max_slots;
    SGN_HIP(hipMemcpyAsync(h_fin + r, fin + r, sizeof(int), hipMemcpyDeviceToHost, s));
    SGN_HIP(hipStreamSynchronize(s));
    if (h_fin[r] != 0) throw SgnError{SGN_EINVAL, "x contains NaN or Inf"};
    Slot& sl = slots[r];
    sl = Slot{};
    sl.busy = true;
    sl.req = next_req++;
    sl.kreq = kreq;
    sl.tol = tol;
    sl.y = y_abi;
    sl.next_ck = first_checkpoint(kreq);
    sl.t0 = std::chrono::steady_clock::now();
    return sl.req;
  }

  // stopping test and next checkpoint of a running slot from its own change
  // history (the rule of sgn_apply, without field-level hints): records the
  // span that ends at k and returns the model's rate
  static double record_span(Slot& sl, int k) {
    if (sl.prev_ck >= 0 && sl.err < 1e29) sl.model.hist.push_back(CkSpan{sl.prev_ck, k, sl.err});
    return sl.model.rate(0.0);
  }
  static int next_checkpoint(Slot& sl, int k, double rate) {
    sl.prev_ck = k;
    return sl.model.next(k, sl.kreq, sl.tol, rate, false);
  }

  // checkpoint (step (v)) for the slots in `due`; finished requests are
  // assembled and recorded.  Returns the number finished.
  int checkpoint(const std::vector<int>& due) {
    hipStream_t s = c->stream;
    Profiler* prof = c->prof.on ? &c->prof : nullptr;
    const bool mixed = prec == SGN_PREC_MIXED;
    const size_t S = (size_t)max_slots, nc = (size_t)ncap, mm = (size_t)std::max(m, 1);
    double* h_err = hpin;
    int* h_flag = reinterpret_cast<int*>(hpin + S);
    double* h_beta = hpin + 2 * S;
    const auto t0 = std::chrono::steady_clock::now();
    SGN_HIP(hipMemcpyAsync(h_flag, flag, sizeof(int) * S, hipMemcpyDeviceToHost, s));
    SGN_HIP(hipStreamSynchronize(s));
    std::map<int, std::vector<int>> groups;  // Krylov dimension -> slots
    std::vector<int> kk(S, 0), brk(S, 0), bad(S, 0);
    for (int r : due) {
      const int f = h_flag[r];
      bad[r] = f < 0;
      brk[r] = f > 0;
      kk[r] = f > 0 ? f - 1 : slots[r].j;
      if (!bad[r]) groups[kk[r]].push_back(r);
    }
    KrylovArgs b0 = base();
    for (auto& g : groups) {
      const int k = g.first, n = m + k, nb = (int)g.second.size();
      const size_t nn = (size_t)n * n;
      double2* Apat = F;
      double2* Fout = F + nn * S;
      if (n > 0) {
        KrylovArgs kc = b0;
        kc.nb = nb;
        for (int z = 0; z < nb; ++z) {
          kc.act[z] = g.second[z];
          kc.jv[z] = k;
        }
        if (k > 0) {
          if (mixed)
            krylov_dot<float2>(kw, kc, false, s, prof);
          else
            krylov_dot<double2>(kw, kc, false, s, prof);
        }
        krylov_patch(kw, kc, n, Apat, nn, k > 0, s);
        const int it = dense_sign_batched(dense, n, nb, Apat, n, nn, Fout, n, nn, s, prof);
        for (int r : g.second) slots[r].newton += std::max(it, 0);
      }
      SlotMap cm;
      cm.n = nb;
      for (int z = 0; z < nb; ++z) {
        cm.slot[z] = g.second[z];
        cm.aux[z] = slots[g.second[z]].nprev;
      }
      dense_coeffs_batched(n, m, Fout, n, nn, c0, (int)mm, beta, cv, cp, (int)nc, cm, err, s);
    }
    SGN_HIP(hipMemcpyAsync(h_err, err, sizeof(double) * S, hipMemcpyDeviceToHost, s));
    SGN_HIP(hipMemcpyAsync(h_beta, beta, sizeof(double) * S, hipMemcpyDeviceToHost, s));
    SGN_HIP(hipStreamSynchronize(s));
    const double ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    int nfinished = 0;
    std::map<int, std::vector<int>> finish;  // ncol -> slots
    for (int r : due) {
      Slot& sl = slots[r];
      sl.ms_sign += ms;
      if (bad[r]) {
        Done d;
        d.status = SGN_EINVAL;
        done[sl.req] = d;
        sl.busy = false;
        ++nfinished;
        continue;
      }
      ++sl.ncheck;
      sl.err = h_err[r];
      sl.nprev = m + kk[r];
      const double rate = record_span(sl, sl.j);
      const bool ok = sl.prev_ck >= 0 && sl.err < 1e29 && CkModel::bound(sl.err, sl.j - sl.prev_ck, rate) <= sl.tol;
      if (brk[r] || ok || sl.j >= sl.kreq) {
        finish[m + kk[r]].push_back(r);
        Done d;
        d.status = (brk[r] || ok) ? SGN_OK : SGN_ENOCONV;
        d.info.k_used = kk[r];
        d.info.converged = (brk[r] || ok) ? 1 : 0;
        d.info.newton_iters = sl.newton;
        d.info.n_matvec = sl.j;
        d.info.n_checkpoints = sl.ncheck;
        d.info.breakdown = brk[r];
        d.info.err_est = sl.err;
        d.info.beta = h_beta[r];
        d.info.ms_sign = sl.ms_sign;
        d.info.ms_total =
            std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - sl.t0).count();
        d.info.ms_arnoldi = d.info.ms_total - sl.ms_sign;
        done[sl.req] = d;
        ++nfinished;
      } else {
        SGN_HIP(hipMemcpyAsync(cp + (size_t)r * nc, cv + (size_t)r * nc, sizeof(double2) * sl.nprev,
                               hipMemcpyDeviceToDevice, s));
        sl.next_ck = next_checkpoint(sl, sl.j, rate);
      }
    }
    // step (vi) for the finished requests: y = Q c into the caller's buffer
    for (auto& g : finish) {
      KrylovArgs kf = b0;
      kf.nb = (int)g.second.size();
      for (int z = 0; z < kf.nb; ++z) kf.act[z] = g.second[z];
      if (mixed)
        krylov_combine<float2>(kw, kf, cv, (int)nc, y, ldq, g.first, s, prof);
      else
        krylov_combine<double2>(kw, kf, cv, (int)nc, y, ldq, g.first, s, prof);
      for (int r : g.second) {
        if (c->lr_m > 0) {  // LR-deflation, step (vi): y += R sgn(Lambda) L^dag x
          double2* lc = lrc + (size_t)r * c->lr_m;
          dev_cmul(c->lrSgn, lc, c->lr_m, s);
          gs_add(gs, c->lrR, ldq, c->N, c->lr_m, lc, y + (size_t)r * ldq, s, prof);
        }
        wilson_unpack(c->lat, y + (size_t)r * ldq, slots[r].y, s);
        slots[r].busy = false;
      }
    }
    if (!finish.empty()) SGN_HIP(hipStreamSynchronize(s));
    return nfinished;
  }

  int step(int nsteps) {
    hipStream_t s = c->stream;
    Profiler* prof = c->prof.on ? &c->prof : nullptr;
    c->prof.stream = s;
    const bool mixed = prec == SGN_PREC_MIXED;
    int nfinished = 0;
    for (int it = 0; it < nsteps; ++it) {
      std::vector<int> active;
      for (int r = 0; r < max_slots; ++r)
        if (slots[r].busy) active.push_back(r);
      if (active.empty()) break;
      KrylovArgs ka = base();
      ka.nb = (int)active.size();
      SlotMap map;
      map.n = ka.nb;
      for (int z = 0; z < ka.nb; ++z) {
        ka.act[z] = active[z];
        ka.jv[z] = slots[active[z]].j;
        map.slot[z] = active[z];
      }
      if (mixed) {
        wilson_apply_slots<float2>(c->lat, c->links32, static_cast<float2*>(ulo), ldq, static_cast<float2*>(z), ldq,
                                   map, s, prof);
        krylov_dot<float2>(kw, ka, true, s, prof);
        krylov_update<float2>(kw, ka, s, prof);
      } else {
        wilson_apply_slots<double2>(c->lat, c->links, u, ldq, static_cast<double2*>(z), ldq, map, s, prof);
        krylov_dot<double2>(kw, ka, true, s, prof);
        krylov_update<double2>(kw, ka, s, prof);
      }
      std::vector<int> due;
      for (int r : active) {
        Slot& sl = slots[r];
        sl.j += 1;
        if (sl.j == sl.next_ck || sl.j >= sl.kreq) due.push_back(r);
      }
      if (!due.empty()) nfinished += checkpoint(due);
    }
    if (prof) c->prof.flush();
    return nfinished;
  }
};

extern "C" {

sgn_session* sgn_session_create(sgn_ctx* c, int max_slots, int kmax) {
  if (!c) return nullptr;
  sgn_session* ss = nullptr;
  const int st = guarded(c, [&] {
    SGN_REQUIRE(max_slots >= 1 && max_slots <= kMaxBatch, SGN_EINVAL, "max_slots must satisfy 1 <= max_slots <= 64");
    SGN_REQUIRE(kmax >= 2 && kmax <= c->N, SGN_EINVAL, "kmax must satisfy 2 <= kmax <= N");
    std::unique_ptr<sgn_session> p(new sgn_session);
    p->c = c;
    p->max_slots = max_slots;
    p->kmax = kmax;
    p->m = c->m;
    p->ncap = c->m + kmax + 1;
    p->prec = c->prec;
    p->ldq = c->ldq;
    p->slots.resize(max_slots);
    try {
      p->alloc();
    } catch (...) {
      p->release();
      throw;
    }
    ss = p.release();
    c->sessions += 1;
    return (int)SGN_OK;
  });
  return st == SGN_OK ? ss : nullptr;
}

int sgn_session_submit(sgn_session* ss, const double* x, double* y, double tol, int kmax, int* req) {
  if (!ss) return SGN_ESTATE;
  return guarded(ss->c, [&] {
    SGN_REQUIRE(req, SGN_EINVAL, "req must not be NULL");
    const int r = ss->submit(reinterpret_cast<const double2*>(x), reinterpret_cast<double2*>(y), tol, kmax);
    if (r < 0) {
      ss->c->last_error = "no free slot in the session";
      return r;
    }
    *req = r;
    return (int)SGN_OK;
  });
}

int sgn_session_step(sgn_session* ss, int nsteps) {
  if (!ss) return SGN_ESTATE;
  return guarded(ss->c, [&] {
    SGN_REQUIRE(nsteps >= 0, SGN_EINVAL, "nsteps must be >= 0");
    return ss->step(nsteps);
  });
}

int sgn_session_poll(sgn_session* ss, int req, sgn_info* info) {
  if (!ss) return SGN_ESTATE;
  return guarded(ss->c, [&] {
    auto it = ss->done.find(req);
    if (it != ss->done.end()) {
      const Done d = it->second;
      ss->done.erase(it);
      if (info) *info = d.info;
      return d.status == SGN_OK || d.status == SGN_ENOCONV ? 1 : d.status;
    }
    for (const auto& sl : ss->slots)
      if (sl.busy && sl.req == req) return 0;
    SGN_REQUIRE(false, SGN_EINVAL, "unknown request (never submitted, or already polled)");
    return (int)SGN_EINVAL;
  });
}

int sgn_session_active(const sgn_session* ss) {
  if (!ss) return SGN_ESTATE;
  int n = 0;
  for (const auto& sl : ss->slots) n += sl.busy ? 1 : 0;
  return n;
}

void sgn_session_destroy(sgn_session* ss) {
  if (!ss) return;
  ss->release();
  ss->c->sessions -= 1;
  delete ss;
}

}  // extern "C"
