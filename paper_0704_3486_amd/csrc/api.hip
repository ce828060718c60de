// C ABI of libsgn: context management and the deflated modified Arnoldi
// driver (Section 5.2, steps (iii)-(vi)) for one source.
//
// Step (iii): pack x, one classical Gram-Schmidt pass against S_m gives
// c0 = S^dag x and x - S c0; its re-orthogonalisation is folded into Arnoldi
// step 0.  Step (iv) (Eq. eq:modArnoldi), per Krylov step j on the device,
// with u the unnormalised candidate of step j (krylov.hip):
//     z = H_w(mu) u                           (stencil)
//     a = Q^dag u, b = Q^dag z, |u|^2, u^dag z (one reduction pass over Q)
//     v_j = (u - Q a) / rho,  u' = (z - g u - Q (b - g a)) / rho
//     column j of H, and a folded into column j-1 (its re-orthogonalisation)
// with Q = (S_m, v_1..v_{j-1}) and rho = |u - Q a|: every new vector is
// orthogonalised twice against all of Q (classical Gram-Schmidt with one
// re-orthogonalisation), in two sweeps over Q per step.  X = S_m^dag A V_k
// and H_k accumulate in one composite matrix H = [[T_m, X], [0, H_k]]
// (Eq. eq:newH).  At even checkpoints k (step (v)) the device evaluates the
// sign of the composite matrix (Newton-Schulz on the matrix cores, Roberts'
// iteration of Eq. Roberts as the fallback), which holds sgn(T_m), sgn(H_k)
// and the Sylvester block Y of Eq. (eq:f_H), then c = sgn(H) Q^dag x with
// Q^dag x = [c0; beta e_1].  Step (vi) is y = Q c (Eq. eq:formula).
// Convergence: ||c_k - [c_k'; 0]|| / ||c_k|| between checkpoints is exactly
// the relative change of y (Q has orthonormal columns); the stopping rule
// (ckpt.h) divides it by the model's 1 - exp(r (k - k')) and certifies the
// earlier checkpoint against tol.
// The two-pass schedule (SGN_ORTH_CGS2: gs.hip, four sweeps per step) is kept
// as an option.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <complex>
#include <cstdint>
#include <cstring>
#include <memory>
#include <mutex>
#include <string>
#include <vector>

#include "ckpt.h"
#include "context.h"

// ---------------------------------------------------------------------------
// profiler
// ---------------------------------------------------------------------------
hipEvent_t Profiler::get_event() {
  if (!pool.empty()) {
    hipEvent_t e = pool.back();
    pool.pop_back();
    return e;
  }
  hipEvent_t e;
  SGN_HIP(hipEventCreate(&e));
  return e;
}

int Profiler::begin(int cls) {
  if (!on) return -1;
  Pending p{get_event(), get_event(), cls};
  SGN_HIP(hipEventRecord(p.a, stream));
  pending.push_back(p);
  return (int)pending.size() - 1;
}

void Profiler::end(int idx, double nbytes, double nflops, int count) {
  if (!on || idx < 0) return;
  Pending& p = pending[idx];
  SGN_HIP(hipEventRecord(p.b, stream));
  launches[p.cls] += count;
  bytes[p.cls] += nbytes;
  flops[p.cls] += nflops;
}

void Profiler::flush() {
  if (pending.empty()) return;
  SGN_HIP(hipStreamSynchronize(stream));
  for (auto& p : pending) {
    float t = 0.f;
    SGN_HIP(hipEventElapsedTime(&t, p.a, p.b));
    ms[p.cls] += t;
    pool.push_back(p.a);
    pool.push_back(p.b);
  }
  pending.clear();
}

void Profiler::reset() {
  for (int i = 0; i < K_NCLASS; ++i) {
    launches[i] = 0;
    ms[i] = bytes[i] = flops[i] = 0.0;
  }
}

Profiler::~Profiler() {
  for (auto& p : pending) {
    (void)hipEventDestroy(p.a);
    (void)hipEventDestroy(p.b);
  }
  for (auto e : pool) (void)hipEventDestroy(e);
}

static const char* kclass_name(int c) {
  switch (c) {
    case K_WILSON: return "wilson_hw";
    case K_KDOT: return "krylov_dot";
    case K_KRED: return "krylov_reduce";
    case K_KUPDATE: return "krylov_update";
    case K_KCOMBINE: return "krylov_combine";
    case K_NS_GEMM: return "ns_gemm";
    case K_GJ_PANEL: return "gj_inverse";
    case K_NEWTON_COMBINE: return "newton_combine";
    case K_CGS_DOT: return "cgs_dot";
    case K_CGS_UPDATE: return "cgs_update";
    case K_BDOT: return "block_dot";
    case K_BRED: return "block_reduce";
    case K_BUPDATE: return "block_update";
    case K_BSMALL: return "block_factor";
    default: return "misc";
  }
}

// Staging of sgn_matvec_noalloc (the packed source and H_w(mu) of it, two
// vectors of the internal layout), for callers that cannot allocate device
// memory.  A file-scope device array: each GPU the library runs on holds its
// own copy until the process ends.  Host code never uses the array's name as
// an address: sgn_create looks up each device's copy once, with that device
// current, and every launch takes the looked-up pointer.
constexpr size_t kScratchBytes = size_t(64) << 20;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

namespace {

std::mutex g_scratch_mu;
std::vector<void*> g_scratch_ptr;   // per device, null until looked up
std::vector<hipError_t> g_scratch_err;

// look up the device copy of `scratch` for device dev (current); once per device
void scratch_lookup(int dev) {
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if ((int)g_scratch_ptr.size() <= dev) {
    g_scratch_ptr.resize(dev + 1, nullptr);
    g_scratch_err.resize(dev + 1, hipSuccess);
  }
  if (g_scratch_ptr[dev] || g_scratch_err[dev] != hipSuccess) return;
  void* p = nullptr;
  const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
  if (e == hipSuccess && p)
    g_scratch_ptr[dev] = p;
  else
    g_scratch_err[dev] = e == hipSuccess ? hipErrorInvalidSymbol : e;
}

void* scratch_device_ptr(int dev) {
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  SGN_REQUIRE(dev >= 0 && dev < (int)g_scratch_ptr.size() && g_scratch_ptr[dev], SGN_EHIP,
              std::string("static staging buffer unavailable on this device: ") +
                  (dev >= 0 && dev < (int)g_scratch_err.size() ? hipGetErrorString(g_scratch_err[dev])
                                                               : "no context was created on it"));
  return g_scratch_ptr[dev];
}

thread_local std::string g_create_error;

int even_up(int k) { return (k + 1) & ~1; }

double elapsed_ms(hipEvent_t a, hipEvent_t b) {
  float t = 0.f;
  SGN_HIP(hipEventElapsedTime(&t, a, b));
  return (double)t;
}

struct EventPair {
  hipEvent_t a = nullptr, b = nullptr;
  EventPair() {
    SGN_HIP(hipEventCreate(&a));
    SGN_HIP(hipEventCreate(&b));
  }
  ~EventPair() {
    if (a) (void)hipEventDestroy(a);
    if (b) (void)hipEventDestroy(b);
  }
};

// Result of the Arnoldi driver.
struct ApplyResult {
  int status = SGN_OK;
};

// One step of the one-reduction Arnoldi recurrence (step (iv)): z = H_w u,
// then the dot and update passes of the argument block.
static void arnoldi_step(sgn_ctx* c, const KrylovArgs& ka, bool mixed, hipStream_t s, Profiler* prof) {
  if (mixed) {
    wilson_apply_multi32(c->lat, c->links32, static_cast<const float2*>(ka.ulonext), 0, c->z32, 0, 1, true, s,
                         prof);
    krylov_dot<float2>(c->kw, ka, true, s, prof);
    krylov_update<float2>(c->kw, ka, s, prof);
  } else {
    wilson_apply(c->lat, c->links, ka.u, c->wB, nullptr, nullptr, s, prof);
    krylov_dot<double2>(c->kw, ka, true, s, prof);
    krylov_update<double2>(c->kw, ka, s, prof);
  }
}

// The graph of L consecutive Arnoldi steps whose step index comes from
// c->jdev (advanced by L at its end), valid for chunks starting at any j in
// the same 32-column bucket of j + L - 1; captured on first use.  It holds
// only kernel launches.
static hipGraphExec_t step_graph(sgn_ctx* c, const KrylovArgs& ka0, bool mixed, int j, int L) {
  const int b = (j + L - 1) / 32;
  if ((int)c->graphs.size() <= b) c->graphs.resize(b + 1, nullptr);
  if (c->graphs[b]) return c->graphs[b];
  // grids sized for the largest step of the bucket
  const int jcap = std::min(32 * (b + 1) - 1, c->kcap - 1);
  SGN_REQUIRE(j + L - 1 <= jcap, SGN_EINVAL, "captured steps exceed the workspace");
  if (!c->cap_stream) SGN_HIP(hipStreamCreateWithFlags(&c->cap_stream, hipStreamNonBlocking));
  hipStream_t cs = c->cap_stream;
  KrylovArgs ka = ka0;
  ka.single(jcap);
  ka.jdev = c->jdev;
  hipGraph_t g = nullptr;
  SGN_HIP(hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal));
  try {
    for (int t = 0; t < L; ++t) {
      ka.joff = t;
      arnoldi_step(c, ka, mixed, cs, nullptr);
    }
    krylov_set_index(c->jdev, L, true, cs);
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
  c->graphs[b] = ex;
  return ex;
}

static int run_apply_impl(sgn_ctx* c, const double2* x_abi, double2* y_abi, double tol, int kmax, int fixed_k,
                          bool allow_block);

// Steps (iii)-(vi).  fixed_k >= 0: exactly that many steps, no convergence test.
int run_apply(sgn_ctx* c, const double2* x_abi, double2* y_abi, double tol, int kmax, int fixed_k) {
  try {
    return run_apply_impl(c, x_abi, y_abi, tol, kmax, fixed_k, true);
  } catch (const BlockFallback&) {
    return run_apply_impl(c, x_abi, y_abi, tol, kmax, fixed_k, false);
  }
}

static int run_apply_impl(sgn_ctx* c, const double2* x_abi, double2* y_abi, double tol, int kmax, int fixed_k,
                          bool allow_block) {
  const auto t_start = std::chrono::steady_clock::now();
  hipStream_t s = c->stream;
  Profiler* prof = c->prof.on ? &c->prof : nullptr;
  c->prof.stream = s;
  const int m = c->m;
  const int N = c->N;
  const size_t ldq = c->ldq;
  const int kwant = fixed_k >= 0 ? fixed_k : kmax;
  c->ensure_workspace(std::max(kwant, 2));
  const int ncap = c->ncap;
  const bool mixed = (c->prec == SGN_PREC_MIXED);
  // block Arnoldi process (FP64 only); else one vector per step
  const bool block = allow_block && !mixed && c->block_s > 0;
  const int sblk = block ? c->block_s : 1;
  const bool delayed = !block && (mixed || c->orth == SGN_ORTH_DELAYED);
  BlockSpan bsp;  // the block process's basis: Q = (S V) in one matrix
  if (block) {
    if (c->blk.ncap < c->ncap || c->blk.nslots < 1) block_alloc(c->blk, N, ldq, c->ncap, 1);
    if (!(c->cheb_e > 0.0)) c->cheb_e = std::sqrt(sq_radius_estimate(c, 40, 0x5eedull));
    SGN_HIP(hipMemsetAsync(c->blk.flag, 0, sizeof(int), s));
    bsp.S = c->Q;
    bsp.V = c->Q + (size_t)m * ldq;
    bsp.ldq = ldq;
    bsp.m = m;
    bsp.N = N;
    bsp.ncap = c->ncap;
    bsp.H = c->Hc;
    bsp.ldh = c->ncap;
    bsp.nb = 1;
  }
  // checkpoints of the block process fall on whole blocks
  auto align = [&](int kk) { return block ? std::min(kmax, (kk + sblk - 1) / sblk * sblk) : kk; };
  sgn_info info{};
  double ms_sign = 0.0;

  // argument block of the one-reduction step (krylov.hip)
  KrylovArgs ka;
  ka.tune = c->tune;
  ka.N = N;
  ka.ldq = ldq;
  ka.m = m;
  ka.S = c->Q;
  ka.V = mixed ? (void*)c->V32 : (void*)(c->Q + (size_t)m * ldq);
  ka.H = c->Hc;
  ka.ldh = ncap;
  ka.c0 = c->c0;
  ka.beta = &c->scal[0];
  ka.flag = c->flag;
  ka.brk_tol = mixed ? 1e-6 : 1e-12;
  // the candidate is updated in place by each step (FP64, and its FP32 copy
  // in mixed precision), so every step's launch arguments are the same
  double2* const ucur = c->wA;
  float2* const u32cur = c->u32a;

  // step (iii): x_perp = (1 - S S^dag) x, beta = |x_perp|
  SGN_HIP(hipMemsetAsync(c->flag, 0, sizeof(int) * 2, s));
  wilson_pack(c->lat, x_abi, c->xin, s);
  dev_check_finite(c->xin, (size_t)N, c->flag + 1, s);
  SGN_HIP(hipMemcpyAsync(c->wA, c->xin, sizeof(double2) * N, hipMemcpyDeviceToDevice, s));
  const int lrm = c->lr_m;
  if (lrm > 0) {
    // LR-deflation, step (iii): L^dag x, and x_- = (1 - R L^dag) x in place of x
    gs_dot(c->gs, c->lrL, ldq, N, lrm, c->wA, c->lrC, s, prof);
    gs_update(c->gs, c->lrR, ldq, N, lrm, c->lrC, c->wA, nullptr, 0, s, prof);
  }
  if (delayed) {
    // one pass against S now; its re-orthogonalisation is folded into step 0
    gs_norm(c->gs, N, c->xin, &c->scal[5], &c->scal[6], nullptr, s, prof);
    SGN_HIP(hipMemcpyAsync(c->kw.sc + kScRef, &c->scal[5], sizeof(double), hipMemcpyDeviceToDevice, s));
    if (m > 0) {
      gs_dot(c->gs, c->Q, ldq, N, m, c->wA, c->c0, s, prof);
      gs_update(c->gs, c->Q, ldq, N, m, c->c0, c->wA, nullptr, 0, s, prof);
    }
    if (mixed) dev_to_f32(c->wA, u32cur, (size_t)N, s);
  } else if (m > 0) {
    gs_dot(c->gs, c->Q, ldq, N, m, c->wA, c->hbuf1, s, prof);
    gs_update(c->gs, c->Q, ldq, N, m, c->hbuf1, c->wA, nullptr, 0, s, prof);
    gs_dot(c->gs, c->Q, ldq, N, m, c->wA, c->hbuf2, s, prof);
    // c0 = h1 + h2 (m entries; the beta slot lands in cvec[m])
    GsFinal fin{c->hbuf1, c->cvec, &c->scal[0], &c->scal[1], c->flag};
    gs_update(c->gs, c->Q, ldq, N, m, c->hbuf2, c->wA, &fin, 0, s, prof);
    SGN_HIP(hipMemcpyAsync(c->c0, c->cvec, sizeof(double2) * m, hipMemcpyDeviceToDevice, s));
  } else {
    gs_norm(c->gs, N, c->wA, &c->scal[0], &c->scal[1], c->flag, s, prof);
  }
  SGN_HIP(hipMemcpyAsync(c->hpin, c->scal, sizeof(double) * 2, hipMemcpyDeviceToHost, s));
  SGN_HIP(hipMemcpyAsync(&c->hpin[4], c->flag, sizeof(int) * 2, hipMemcpyDeviceToHost, s));
  SGN_HIP(hipStreamSynchronize(s));
  int hflag[2];
  std::memcpy(hflag, &c->hpin[4], sizeof(int) * 2);
  if (hflag[1] != 0 || hflag[0] < 0) throw SgnError{SGN_EINVAL, "x contains NaN or Inf"};
  // the two-pass schedule knows x_perp already; the delayed one finds x_perp = 0
  // as a breakdown of step 0
  const bool x_in_schur = !delayed && (hflag[0] == 1);

  int k = 0;
  bool converged = false;
  bool breakdown = false;
  int nprev = -1;  // size of cprev (m + k') or -1
  double err = 1e30;
  int ncheck = 0;
  int newton_total = 0;
  CkModel model;  // changes between checkpoints (placement and stopping rule)
  int prev_ck = -1;

  auto checkpoint = [&](int kk) -> double {
    // sign of the composite (m + kk) matrix, coefficients, change estimate
    const int n = m + kk;
    const auto t0 = std::chrono::steady_clock::now();
    int it = 0;
    if (n > 0) {
      if (delayed && kk > 0) {
        // finish the re-orthogonalisation of the last column, on a copy
        ka.single(kk);
        ka.u = ucur;
        if (mixed)
          krylov_dot<float2>(c->kw, ka, false, s, prof);
        else
          krylov_dot<double2>(c->kw, ka, false, s, prof);
        krylov_patch(c->kw, ka, n, c->F, 0, true, s);
        it = dense_sign(c->dense, n, c->F, n, c->F, n, s, prof, c->cheb_e);
      } else {
        it = dense_sign(c->dense, n, c->Hc, ncap, c->F, n, s, prof, c->cheb_e);
      }
    }
    newton_total += it;
    dense_coeffs(n, m, c->F, n, c->c0, &c->scal[0], c->cvec, nprev >= 0 ? c->cprev : nullptr,
                 nprev >= 0 ? nprev : 0, &c->scal[2], s);
    SGN_HIP(hipMemcpyAsync(&c->hpin[2], &c->scal[2], sizeof(double), hipMemcpyDeviceToHost, s));
    SGN_HIP(hipStreamSynchronize(s));
    ms_sign += std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    ++ncheck;
    const double e = c->hpin[2];
    SGN_HIP(hipMemcpyAsync(c->cprev, c->cvec, sizeof(double2) * n, hipMemcpyDeviceToDevice, s));
    nprev = n;
    return e;
  };

  if (x_in_schur || kwant == 0) {
    // y = S sgn(T) S^dag x exactly (no Krylov part), or k = 0 requested
    SGN_HIP(hipMemsetAsync(&c->scal[0], 0, sizeof(double), s));
    if (m > 0) err = checkpoint(0);
    converged = true;
    breakdown = x_in_schur;
  } else {
    // Krylov loop (step (iv)) with checkpoints (step (v))
    // First checkpoint: where the previous apply on this field certified
    // convergence (its last-but-one checkpoint), else 32.  This only moves the
    // checkpoints; the stopping test is the same.
    int next_ck;
    const bool hinted = c->k_hint > 0 && c->tol_hint == tol;
    if (fixed_k >= 0) {
      next_ck = fixed_k;
    } else if (hinted) {
      next_ck = align(std::min(kmax, std::max(2, even_up(c->k_hint))));
    } else {
      next_ck = align(std::min(kmax, std::max(2, even_up(std::min(32, kmax / 2)))));
    }
    double2* wprev = c->wA;  // two-pass schedule: x_perp (unnormalised) for j = 0
    double2* wcur = c->wB;
    ka.u = ucur;
    ka.unext = ucur;
    ka.z = mixed ? (const void*)c->z32 : (const void*)c->wB;
    ka.ulonext = mixed ? (void*)u32cur : nullptr;
    for (int j = 0; j < kwant;) {
      const int J = m + j;
      const int seg_end = std::min(next_ck, kwant);  // the next checkpoint
      const int L = c->graph_steps;
      if (delayed && !prof && L > 0 && j + L <= seg_end) {
        // whole captured chunks of L steps up to the checkpoint
        krylov_set_index(c->jdev, j, false, s);
        while (j + L <= seg_end) {
          SGN_HIP(hipGraphLaunch(step_graph(c, ka, mixed, j, L), s));
          j += L;
          info.n_matvec += L;
        }
      } else if (delayed) {
        ka.single(j);
        arnoldi_step(c, ka, mixed, s, prof);
        ++j;
        info.n_matvec += 1;
      } else if (block) {
        const int sb = std::min(sblk, seg_end - j);
        if (j == 0) block_first(bsp, c->wA, 0, &c->scal[1], 0, s);  // v_1 = x_perp / beta
        block_step(bsp, c->blk, c->lat, c->links, j, sb, c->cheb_e, s, prof);
        j += sb;
        info.n_matvec += sb;
      } else {
        double2* vcol = c->Q + (size_t)J * ldq;
        wilson_apply(c->lat, c->links, wprev, wcur, &c->scal[1], vcol, s, prof);
        const int ncol = J + 1;
        gs_dot(c->gs, c->Q, ldq, N, ncol, wcur, c->hbuf1, s, prof);
        gs_update(c->gs, c->Q, ldq, N, ncol, c->hbuf1, wcur, nullptr, 0, s, prof);
        gs_dot(c->gs, c->Q, ldq, N, ncol, wcur, c->hbuf2, s, prof);
        GsFinal fin{c->hbuf1, c->Hc + (size_t)J * ncap, nullptr, &c->scal[1], c->flag};
        gs_update(c->gs, c->Q, ldq, N, ncol, c->hbuf2, wcur, &fin, j + 1, s, prof);
        std::swap(wprev, wcur);
        ++j;
        info.n_matvec += 1;
      }
      k = j;
      if (k == next_ck || k == kwant) {
        // breakdown check (flag = k_invariant + 1)
        SGN_HIP(hipMemcpyAsync(&c->hpin[4], c->flag, sizeof(int), hipMemcpyDeviceToHost, s));
        SGN_HIP(hipStreamSynchronize(s));
        int f0;
        std::memcpy(&f0, &c->hpin[4], sizeof(int));
        if (block) {
          SGN_HIP(hipMemcpyAsync(&c->hpin[4], c->blk.flag, sizeof(int), hipMemcpyDeviceToHost, s));
          SGN_HIP(hipStreamSynchronize(s));
          int bf;
          std::memcpy(&bf, &c->hpin[4], sizeof(int));
          if (bf != 0) throw BlockFallback{};
        }
        if (f0 < 0) throw SgnError{SGN_EINVAL, "non-finite value in the Krylov basis"};
        if (f0 > 0) {
          k = f0 - 1;
          breakdown = true;
        }
        const double e = checkpoint(k);
        if (fixed_k >= 0 || breakdown) {
          err = e;
          converged = true;
          break;
        }
        if (prev_ck >= 0 && e < 1e29) model.hist.push_back(CkSpan{prev_ck, k, e});
        err = e;
        // rate of the geometric error model: from this apply's last two
        // spans, else from the first apply on this field
        const double rate = model.rate(c->rate_hint < 0.0 ? c->rate_hint : 0.0);
        if (model.hist.size() >= 2 && CkModel::usable(rate) && c->rate_hint == 0.0) c->rate_hint = rate;
        if (prev_ck >= 0 && e < 1e29 && CkModel::bound(e, k - prev_ck, rate) <= tol) {
          converged = true;
          // the previous checkpoint is certified: remember it (once per
          // field, so later applies share one schedule)
          if (c->k_hint == 0) {
            c->k_hint = prev_ck;
            c->tol_hint = tol;
          }
          break;
        }
        prev_ck = k;
        next_ck = align(model.next(k, kmax, tol, rate, hinted && model.hist.empty()));
      }
    }
  }

  // step (vi): y = Q c
  const int n = m + k;
  if (delayed || block) {
    if (mixed)
      krylov_combine<float2>(c->kw, ka, c->cvec, 0, c->wB, 0, n, s, prof);
    else
      krylov_combine<double2>(c->kw, ka, c->cvec, 0, c->wB, 0, n, s, prof);
  } else {
    gs_combine(c->gs, c->Q, ldq, N, n, c->cvec, c->wB, nullptr, s, prof);
  }
  if (lrm > 0) {
    // LR-deflation, step (vi): y += R sgn(Lambda) L^dag x
    dev_cmul(c->lrSgn, c->lrC, lrm, s);
    gs_add(c->gs, c->lrR, ldq, N, lrm, c->lrC, c->wB, s, prof);
  }
  wilson_unpack(c->lat, c->wB, y_abi, s);
  SGN_HIP(hipMemcpyAsync(&c->hpin[6], &c->scal[0], sizeof(double), hipMemcpyDeviceToHost, s));
  SGN_HIP(hipStreamSynchronize(s));
  if (prof) c->prof.flush();
  info.beta = c->hpin[6];

  info.k_used = k;
  info.converged = converged ? 1 : 0;
  info.newton_iters = newton_total;
  info.n_checkpoints = ncheck;
  info.breakdown = breakdown ? 1 : 0;
  info.err_est = err;
  info.ms_sign = ms_sign;
  info.ms_total =
      std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t_start).count();
  info.ms_arnoldi = info.ms_total - ms_sign;
  c->info = info;
  if (fixed_k < 0 && !converged) {
    c->last_error = "kmax reached before the requested tolerance";
    return SGN_ENOCONV;
  }
  return SGN_OK;
}

}  // namespace

void install_schur_pair(sgn_ctx* c, int m, const double2* S_internal, const std::vector<double2>& Tin) {
  SGN_REQUIRE(c->sessions == 0, SGN_ESTATE, "a serving session holds this field's Schur pair");
  hipStream_t s = c->stream;
  SGN_HIP(hipStreamSynchronize(s));
  std::vector<double2> Th(Tin);
  for (int j = 0; j < m; ++j)
    for (int i = j + 1; i < m; ++i) Th[(size_t)j * m + i] = make_double2(0.0, 0.0);
  for (int i = 0; i < m; ++i) {
    const double2 d = Th[(size_t)i * m + i];
    SGN_REQUIRE(std::isfinite(d.x) && std::isfinite(d.y), SGN_EINVAL, "T has a non-finite diagonal");
    SGN_REQUIRE(d.x != 0.0, SGN_ESINGULAR, "T has an eigenvalue on the imaginary axis");
  }
  // drop the old basis (Schur or LR) and the workspaces (their layout depends on m)
  c->drop_lr();
  c->release_workspace();
  c->bw.release();
  c->bw.k_hint = 0;
  c->bw.rate_hint = 0.0;
  for (double2** p : {&c->S, &c->Tdev, &c->sgnT})
    if (*p) {
      SGN_HIP(hipFree(*p));
      *p = nullptr;
    }
  c->T.clear();
  c->m = 0;
  if (m == 0) return;
  SGN_HIP(hipMalloc(&c->S, sizeof(double2) * c->ldq * (size_t)m));
  SGN_HIP(hipMemcpyAsync(c->S, S_internal, sizeof(double2) * c->ldq * (size_t)m, hipMemcpyDeviceToDevice, s));
  SGN_HIP(hipMalloc(&c->Tdev, sizeof(double2) * (size_t)m * m));
  SGN_HIP(hipMalloc(&c->sgnT, sizeof(double2) * (size_t)m * m));
  SGN_HIP(hipMemcpyAsync(c->Tdev, Th.data(), sizeof(double2) * Th.size(), hipMemcpyHostToDevice, s));
  dense_sign(c->dense, m, c->Tdev, m, c->sgnT, m, s, nullptr);  // step (ii): sgn(T_m)
  SGN_HIP(hipStreamSynchronize(s));
  c->T = std::move(Th);
  c->m = m;
  c->k_hint = 0;
  c->rate_hint = 0.0;
}

// Install an LR-deflation pair (the LR-deflation subsection, steps (i)-(ii)):
// right and left eigenvectors in the internal layout (device, ldq x m) with
// L^dag R = I, and the eigenvalues (host).  Replaces any Schur pair (m = 0
// for the Krylov part).
void install_lr_pair(sgn_ctx* c, int m, const double2* R_internal, const double2* L_internal,
                     const std::vector<double2>& lam) {
  install_schur_pair(c, 0, nullptr, {});
  if (m == 0) return;
  hipStream_t s = c->stream;
  std::vector<double2> sg((size_t)m);
  for (int i = 0; i < m; ++i) {
    SGN_REQUIRE(std::isfinite(lam[i].x) && std::isfinite(lam[i].y), SGN_EINVAL, "non-finite eigenvalue");
    SGN_REQUIRE(lam[i].x != 0.0, SGN_ESINGULAR, "an eigenvalue lies on the imaginary axis");
    sg[i] = make_double2(lam[i].x > 0.0 ? 1.0 : -1.0, 0.0);  // step (ii): sgn(lambda_i) = sgn(Re lambda_i)
  }
  try {
    SGN_HIP(hipMalloc(&c->lrR, sizeof(double2) * c->ldq * (size_t)m));
    SGN_HIP(hipMalloc(&c->lrL, sizeof(double2) * c->ldq * (size_t)m));
    SGN_HIP(hipMalloc(&c->lrSgn, sizeof(double2) * (size_t)m));
    SGN_HIP(hipMalloc(&c->lrC, sizeof(double2) * (size_t)m));
    SGN_HIP(hipMemcpyAsync(c->lrR, R_internal, sizeof(double2) * c->ldq * (size_t)m, hipMemcpyDeviceToDevice, s));
    SGN_HIP(hipMemcpyAsync(c->lrL, L_internal, sizeof(double2) * c->ldq * (size_t)m, hipMemcpyDeviceToDevice, s));
    SGN_HIP(hipMemcpyAsync(c->lrSgn, sg.data(), sizeof(double2) * (size_t)m, hipMemcpyHostToDevice, s));
    SGN_HIP(hipStreamSynchronize(s));
  } catch (...) {
    c->drop_lr();
    throw;
  }
  c->lrLam = lam;
  c->lr_m = m;
}

// ---------------------------------------------------------------------------
// ABI
// ---------------------------------------------------------------------------
extern "C" {

const char* sgn_strerror(int st) {
  switch (st) {
    case SGN_OK: return "ok";
    case SGN_EINVAL: return "invalid argument";
    case SGN_ENOMEM: return "out of memory";
    case SGN_EHIP: return "HIP runtime error";
    case SGN_ENOCONV: return "not converged within kmax";
    case SGN_ESINGULAR: return "singular matrix or eigenvalue on the imaginary axis";
    case SGN_ESTATE: return "invalid state";
    case SGN_EDEFL: return "deflation basis not accurate enough";
    default: return "unknown status";
  }
}

const char* sgn_create_error(void) { return g_create_error.c_str(); }

const char* sgn_last_error(const sgn_ctx* c) { return c ? c->last_error.c_str() : "null context"; }

sgn_ctx* sgn_create(const double* gauge, const int dims[4], double mu, double m_w) {
  g_create_error.clear();
  if (!gauge || !dims) {
    g_create_error = "gauge and dims must not be NULL";
    return nullptr;
  }
  for (int d = 0; d < 4; ++d)
    if (dims[d] < 2) {
      g_create_error = "every lattice extent must be >= 2";
      return nullptr;
    }
  if (!(8.0 + 2.0 * m_w > 0.0) || !std::isfinite(mu) || !std::isfinite(m_w)) {
    g_create_error = "need 8 + 2 m_w > 0 and finite mu, m_w";
    return nullptr;
  }
  const long long V = (long long)dims[0] * dims[1] * dims[2] * dims[3];
  if (V * 12 > (1LL << 30)) {
    g_create_error = "lattice too large";
    return nullptr;
  }
  std::unique_ptr<sgn_ctx> c(new (std::nothrow) sgn_ctx());
  if (!c) {
    g_create_error = "host allocation failed";
    return nullptr;
  }
  try {
    for (int d = 0; d < 4; ++d) c->lat.L[d] = dims[d];
    c->lat.V = (int)V;
    c->lat.kappa = 1.0 / (8.0 + 2.0 * m_w);
    c->lat.emu = std::exp(mu);
    c->lat.emmu = std::exp(-mu);
    c->mu = mu;
    c->m_w = m_w;
    c->N = (int)(12 * V);
    c->ldq = ((size_t)c->N + 63) / 64 * 64;
    SGN_HIP(hipGetDevice(&c->device));
    scratch_lookup(c->device);  // once per device (sgn_matvec_noalloc)
    SGN_HIP(hipMalloc(&c->links, sizeof(double2) * wilson_link_entries((int)V)));
    SGN_HIP(hipMalloc(&c->scal, sizeof(double) * 8));
    SGN_HIP(hipMalloc(&c->flag, sizeof(int) * 4));
    SGN_HIP(hipHostMalloc(&c->hpin, sizeof(double) * 8, hipHostMallocDefault));
    SGN_HIP(hipMemset(c->scal, 0, sizeof(double) * 8));
    SGN_HIP(hipMemset(c->flag, 0, sizeof(int) * 4));
    double2* graw = nullptr;
    SGN_HIP(hipMalloc(&graw, sizeof(double2) * 36 * (size_t)V));
    SGN_HIP(hipMemcpy(graw, gauge, sizeof(double2) * 36 * (size_t)V, hipMemcpyHostToDevice));
    wilson_pack_links(c->lat, graw, c->links, c->flag, nullptr);
    SGN_HIP(hipDeviceSynchronize());
    SGN_HIP(hipFree(graw));
    int bad = 0;
    SGN_HIP(hipMemcpy(&bad, c->flag, sizeof(int), hipMemcpyDeviceToHost));
    SGN_HIP(hipMemset(c->flag, 0, sizeof(int) * 4));
    if (bad) {
      g_create_error = "gauge links must be SU(3) (unitary with determinant 1, to 1e-10)";
      return nullptr;
    }
  } catch (const SgnError& e) {
    g_create_error = e.msg;
    return nullptr;
  }
  return c.release();
}

void sgn_destroy(sgn_ctx* c) { delete c; }

int sgn_set_stream(sgn_ctx* c, void* stream) {
  return guarded(c, [&] {
    SGN_HIP(hipDeviceSynchronize());
    c->stream = (hipStream_t)stream;
    c->prof.stream = c->stream;
    return SGN_OK;
  });
}

int sgn_get_dims(const sgn_ctx* c, int dims[4], long long* n) {
  if (!c) return SGN_ESTATE;
  if (dims)
    for (int d = 0; d < 4; ++d) dims[d] = c->lat.L[d];
  if (n) *n = c->N;
  return SGN_OK;
}

int sgn_deflation_size(const sgn_ctx* c) { return c ? (c->lr_m > 0 ? c->lr_m : c->m) : SGN_ESTATE; }

int sgn_deflation_mode(const sgn_ctx* c) {
  if (!c) return SGN_ESTATE;
  return c->lr_m > 0 ? SGN_DEFL_LR : (c->m > 0 ? SGN_DEFL_SCHUR : SGN_DEFL_NONE);
}

int sgn_deflate_lr_import(sgn_ctx* c, int m, const double* R_abi, const double* L_abi, const double* lam_host) {
  return guarded(c, [&] {
    SGN_REQUIRE(m >= 1 && m <= c->N / 4, SGN_EINVAL, "m must satisfy 1 <= m <= N/4");
    SGN_REQUIRE(R_abi && L_abi && lam_host, SGN_EINVAL, "R, L and lam must not be NULL");
    SGN_REQUIRE(c->sessions == 0, SGN_ESTATE, "a serving session holds this field's deflation");
    hipStream_t s = c->stream;
    const size_t ldq = c->ldq;
    std::vector<double2> lam((size_t)m);
    std::memcpy(lam.data(), lam_host, sizeof(double2) * (size_t)m);
    double2 *Rint = nullptr, *Lint = nullptr, *G = nullptr;
    GsWork g;
    try {
      SGN_HIP(hipMalloc(&Rint, sizeof(double2) * ldq * (size_t)m));
      SGN_HIP(hipMalloc(&Lint, sizeof(double2) * ldq * (size_t)m));
      SGN_HIP(hipMalloc(&G, sizeof(double2) * (size_t)m * m));
      SGN_HIP(hipMemsetAsync(Rint, 0, sizeof(double2) * ldq * (size_t)m, s));
      SGN_HIP(hipMemsetAsync(Lint, 0, sizeof(double2) * ldq * (size_t)m, s));
      for (int j = 0; j < m; ++j) {
        wilson_pack(c->lat, reinterpret_cast<const double2*>(R_abi) + (size_t)j * c->N, Rint + (size_t)j * ldq, s);
        wilson_pack(c->lat, reinterpret_cast<const double2*>(L_abi) + (size_t)j * c->N, Lint + (size_t)j * ldq, s);
      }
      // L^dag R = I is required (the oblique projector R L^dag)
      gs_alloc(g, c->N, ldq, m);
      for (int j = 0; j < m; ++j) gs_dot(g, Lint, ldq, c->N, m, Rint + (size_t)j * ldq, G + (size_t)j * m, s, nullptr);
      std::vector<double2> Gh((size_t)m * m);
      SGN_HIP(hipMemcpyAsync(Gh.data(), G, sizeof(double2) * Gh.size(), hipMemcpyDeviceToHost, s));
      SGN_HIP(hipStreamSynchronize(s));
      double dev = 0.0;
      for (int j = 0; j < m; ++j)
        for (int i = 0; i < m; ++i) {
          const double2 e = Gh[(size_t)j * m + i];
          dev = std::max(dev, std::hypot(e.x - (i == j ? 1.0 : 0.0), e.y));
        }
      SGN_REQUIRE(std::isfinite(dev) && dev <= 1e-8, SGN_EINVAL, "L^dag R must equal I (deviation " +
                                                                     std::to_string(dev) + ")");
      install_lr_pair(c, m, Rint, Lint, lam);
    } catch (...) {
      gs_free(g);
      for (double2* p : {Rint, Lint, G})
        if (p) (void)hipFree(p);
      throw;
    }
    gs_free(g);
    for (double2* p : {Rint, Lint, G})
      if (p) SGN_HIP(hipFree(p));
    return SGN_OK;
  });
}

int sgn_deflate_lr_export(const sgn_ctx* cc, double* R_abi, double* L_abi, double* lam_host) {
  sgn_ctx* c = const_cast<sgn_ctx*>(cc);
  return guarded(c, [&] {
    const int m = c->lr_m;
    SGN_REQUIRE(m > 0, SGN_ESTATE, "no LR-deflation pair installed");
    for (int j = 0; j < m; ++j) {
      if (R_abi)
        wilson_unpack(c->lat, c->lrR + (size_t)j * c->ldq, reinterpret_cast<double2*>(R_abi) + (size_t)j * c->N,
                      c->stream);
      if (L_abi)
        wilson_unpack(c->lat, c->lrL + (size_t)j * c->ldq, reinterpret_cast<double2*>(L_abi) + (size_t)j * c->N,
                      c->stream);
    }
    SGN_HIP(hipStreamSynchronize(c->stream));
    if (lam_host) std::memcpy(lam_host, c->lrLam.data(), sizeof(double2) * (size_t)m);
    return SGN_OK;
  });
}

int sgn_deflate_import(sgn_ctx* c, int m, const double* S_abi, const double* T_host) {
  return guarded(c, [&] {
    SGN_REQUIRE(m >= 0 && m <= c->N / 4, SGN_EINVAL, "m must satisfy 0 <= m <= N/4");
    SGN_REQUIRE(m == 0 || (S_abi && T_host), SGN_EINVAL, "S and T must not be NULL");
    std::vector<double2> Th((size_t)m * m);
    if (m) std::memcpy(Th.data(), T_host, sizeof(double2) * Th.size());
    double2* Sint = nullptr;
    if (m) {
      SGN_HIP(hipMalloc(&Sint, sizeof(double2) * c->ldq * (size_t)m));
      SGN_HIP(hipMemsetAsync(Sint, 0, sizeof(double2) * c->ldq * (size_t)m, c->stream));
      for (int j = 0; j < m; ++j)
        wilson_pack(c->lat, reinterpret_cast<const double2*>(S_abi) + (size_t)j * c->N, Sint + (size_t)j * c->ldq,
                    c->stream);
    }
    try {
      install_schur_pair(c, m, Sint, Th);
    } catch (...) {
      if (Sint) (void)hipFree(Sint);
      throw;
    }
    if (Sint) SGN_HIP(hipFree(Sint));
    return SGN_OK;
  });
}

int sgn_deflate_export(const sgn_ctx* cc, double* S_abi, double* T_host, double* evals) {
  sgn_ctx* c = const_cast<sgn_ctx*>(cc);
  return guarded(c, [&] {
    const int m = c->m;
    if (S_abi)
      for (int j = 0; j < m; ++j)
        wilson_unpack(c->lat, c->S + (size_t)j * c->ldq, reinterpret_cast<double2*>(S_abi) + (size_t)j * c->N,
                      c->stream);
    SGN_HIP(hipStreamSynchronize(c->stream));
    if (T_host && m) std::memcpy(T_host, c->T.data(), sizeof(double2) * (size_t)m * m);
    if (evals)
      for (int i = 0; i < m; ++i) {
        evals[2 * i] = c->T[(size_t)i * m + i].x;
        evals[2 * i + 1] = c->T[(size_t)i * m + i].y;
      }
    return SGN_OK;
  });
}

int sgn_apply(sgn_ctx* c, const double* x, double* y, double tol, int kmax) {
  return guarded(c, [&] {
    SGN_REQUIRE(x && y, SGN_EINVAL, "x and y must not be NULL");
    SGN_REQUIRE(tol > 0.0 && std::isfinite(tol), SGN_EINVAL, "tol must be positive");
    SGN_REQUIRE(kmax >= 2 && kmax <= c->N, SGN_EINVAL, "kmax must satisfy 2 <= kmax <= N");
    return run_apply(c, reinterpret_cast<const double2*>(x), reinterpret_cast<double2*>(y), tol, kmax, -1);
  });
}

// [a, a + n) and [b, b + n) (complex entries) share memory
static bool overlapping(const double* a, const double* b, size_t n) {
  const auto pa = reinterpret_cast<uintptr_t>(a), pb = reinterpret_cast<uintptr_t>(b);
  const uintptr_t len = n * sizeof(double2);
  return pa < pb + len && pb < pa + len;
}

int sgn_overlap_apply(sgn_ctx* c, const double* x, double* y, double tol, int kmax) {
  return guarded(c, [&] {
    SGN_REQUIRE(x && y, SGN_EINVAL, "x and y must not be NULL");
    SGN_REQUIRE(!overlapping(x, y, (size_t)c->N), SGN_EINVAL, "x and y must not overlap");
    SGN_REQUIRE(tol > 0.0 && std::isfinite(tol), SGN_EINVAL, "tol must be positive");
    SGN_REQUIRE(kmax >= 2 && kmax <= c->N, SGN_EINVAL, "kmax must satisfy 2 <= kmax <= N");
    const int st = run_apply(c, reinterpret_cast<const double2*>(x), reinterpret_cast<double2*>(y), tol, kmax, -1);
    overlap_finish(reinterpret_cast<const double2*>(x), reinterpret_cast<double2*>(y), (size_t)c->N, c->stream);
    SGN_HIP(hipStreamSynchronize(c->stream));
    return st;
  });
}

int sgn_apply_fixed(sgn_ctx* c, const double* x, double* y, int k) {
  return guarded(c, [&] {
    SGN_REQUIRE(x && y, SGN_EINVAL, "x and y must not be NULL");
    SGN_REQUIRE(k >= 0 && k <= c->N - c->m - c->lr_m, SGN_EINVAL,
                "k must satisfy 0 <= k <= N - (deflation size)");
    return run_apply(c, reinterpret_cast<const double2*>(x), reinterpret_cast<double2*>(y), 1.0, k, k);
  });
}

static int run_adjoint(sgn_ctx* c, const double* x, double* y, double tol, int kmax, int fixed_k) {
  check_adjoint(c);
  AdjointScope scope(c);
  return run_apply(c, reinterpret_cast<const double2*>(x), reinterpret_cast<double2*>(y), tol, kmax, fixed_k);
}

int sgn_apply_adjoint(sgn_ctx* c, const double* x, double* y, double tol, int kmax) {
  return guarded(c, [&] {
    SGN_REQUIRE(x && y, SGN_EINVAL, "x and y must not be NULL");
    SGN_REQUIRE(tol > 0.0 && std::isfinite(tol), SGN_EINVAL, "tol must be positive");
    SGN_REQUIRE(kmax >= 2 && kmax <= c->N, SGN_EINVAL, "kmax must satisfy 2 <= kmax <= N");
    return run_adjoint(c, x, y, tol, kmax, -1);
  });
}

int sgn_apply_adjoint_fixed(sgn_ctx* c, const double* x, double* y, int k) {
  return guarded(c, [&] {
    SGN_REQUIRE(x && y, SGN_EINVAL, "x and y must not be NULL");
    SGN_REQUIRE(k >= 0 && k <= c->N - c->m - c->lr_m, SGN_EINVAL,
                "k must satisfy 0 <= k <= N - (deflation size)");
    return run_adjoint(c, x, y, 1.0, k, k);
  });
}

int sgn_overlap_apply_adjoint(sgn_ctx* c, const double* x, double* y, double tol, int kmax) {
  return guarded(c, [&] {
    SGN_REQUIRE(x && y, SGN_EINVAL, "x and y must not be NULL");
    SGN_REQUIRE(!overlapping(x, y, (size_t)c->N), SGN_EINVAL, "x and y must not overlap");
    SGN_REQUIRE(tol > 0.0 && std::isfinite(tol), SGN_EINVAL, "tol must be positive");
    SGN_REQUIRE(kmax >= 2 && kmax <= c->N, SGN_EINVAL, "kmax must satisfy 2 <= kmax <= N");
    check_adjoint(c);  // before y is written
    const auto x2 = reinterpret_cast<const double2*>(x);
    const auto y2 = reinterpret_cast<double2*>(y);
    overlap_adjoint_start(x2, y2, (size_t)c->N, c->stream);  // y = gamma5 x
    const int st = run_adjoint(c, y, y, tol, kmax, -1);      // y = sgn^dag y (in place)
    overlap_adjoint_finish(x2, y2, (size_t)c->N, c->stream);
    SGN_HIP(hipStreamSynchronize(c->stream));
    return st;
  });
}

// Device buffer owned by one call
struct CallBuf {
  void* p = nullptr;
  explicit CallBuf(size_t bytes) { SGN_HIP(hipMalloc(&p, bytes)); }
  ~CallBuf() {
    if (p) (void)hipFree(p);
  }
  CallBuf(const CallBuf&) = delete;
  CallBuf& operator=(const CallBuf&) = delete;
  double2* c2() const { return static_cast<double2*>(p); }
  double* d() const { return static_cast<double*>(p); }
};

// D(m) x = b for D(m) = (1 - m/2) D_ov(mu) + m = (1 + m/2) + (1 - m/2) gamma5
// sgn(H_w(mu)) (a reading: the paper leaves the inversion of the overlap
// operator to future work, where every outer step needs one sign apply) by
// restarted GMRES.  The outer basis W is orthogonalised with classical
// Gram-Schmidt and one re-orthogonalisation on the device; the small least
// squares problem (Givens rotations) is solved on the host; at each restart
// the true residual b - D x is formed.
int sgn_overlap_solve(sgn_ctx* c, const double* b, double* x, double mass, double tol, int max_iter, int restart,
                      double inner_tol, int inner_kmax, int* iters, double* rel_res) {
  return guarded(c, [&] {
    using cplx = std::complex<double>;
    const int N = c->N;
    SGN_REQUIRE(b && x, SGN_EINVAL, "b and x must not be NULL");
    SGN_REQUIRE(!overlapping(b, x, (size_t)N), SGN_EINVAL, "b and x must not overlap");
    SGN_REQUIRE(mass >= 0.0 && std::isfinite(mass), SGN_EINVAL, "mass must be finite and >= 0");
    SGN_REQUIRE(tol > 0.0 && std::isfinite(tol), SGN_EINVAL, "tol must be positive");
    SGN_REQUIRE(max_iter >= 1, SGN_EINVAL, "max_iter must be >= 1");
    SGN_REQUIRE(restart >= 1 && restart <= 500, SGN_EINVAL, "restart must satisfy 1 <= restart <= 500");
    SGN_REQUIRE(inner_tol > 0.0 && std::isfinite(inner_tol), SGN_EINVAL, "inner_tol must be positive");
    SGN_REQUIRE(inner_kmax >= 2 && inner_kmax <= N, SGN_EINVAL, "inner_kmax must satisfy 2 <= inner_kmax <= N");
    hipStream_t s = c->stream;
    const size_t ld = c->ldq;
    const int R = restart;
    CallBuf bW(sizeof(double2) * ld * (size_t)(R + 1)), bt(sizeof(double2) * ld);
    CallBuf bh(sizeof(double2) * 3 * (size_t)(R + 2)), bsc(sizeof(double) * 4);
    double2* W = bW.c2();
    double2* t = bt.c2();
    double2* h1 = bh.c2();
    double2* h2 = h1 + (R + 2);
    double2* hout = h2 + (R + 2);  // also the solution coefficients y
    double* sc = bsc.d();
    int* dflag = reinterpret_cast<int*>(sc + 2);  // non-finite record of the outer Gram-Schmidt
    GsWork g;
    gs_alloc(g, N, ld, R + 1);
    struct GsGuard {
      GsWork& g;
      ~GsGuard() { gs_free(g); }
    } guard{g};
    const auto b2 = reinterpret_cast<const double2*>(b);
    const auto x2 = reinterpret_cast<double2*>(x);
    const double ca = 1.0 + 0.5 * mass, cb = 1.0 - 0.5 * mass;
    auto apply_D = [&](const double2* v, double2* out) {  // out = D(m) v, out != v
      const int st = run_apply(c, v, out, inner_tol, inner_kmax, -1);
      SGN_REQUIRE(st == SGN_OK, SGN_ENOCONV, "overlap solve: a sign apply did not reach inner_tol within inner_kmax");
      axpby_abi(v, out, ca, cb, true, (size_t)N, s);
    };
    auto norm = [&](const double2* v) {
      gs_norm(g, N, v, &sc[0], &sc[1], nullptr, s, nullptr);
      double r = 0.0;
      SGN_HIP(hipMemcpyAsync(&r, &sc[0], sizeof(double), hipMemcpyDeviceToHost, s));
      SGN_HIP(hipStreamSynchronize(s));
      return r;
    };
    dev_zero(x2, (size_t)N, s);
    const double bnorm = norm(b2);
    SGN_REQUIRE(std::isfinite(bnorm), SGN_EINVAL, "b contains NaN or Inf");
    int it = 0;
    double res = 0.0;
    if (bnorm > 0.0) {
      std::vector<cplx> H((size_t)(R + 1) * R), sn(R), gv(R + 1), y(R);
      std::vector<double> cs(R);
      std::vector<double2> hh(R + 2);
      for (bool first = true;; first = false) {
        // true residual r = b - D x in W_0
        if (first) {
          SGN_HIP(hipMemcpyAsync(W, b2, sizeof(double2) * N, hipMemcpyDeviceToDevice, s));
        } else {
          apply_D(x2, t);
          axpby_abi(b2, t, 1.0, -1.0, false, (size_t)N, s);
          SGN_HIP(hipMemcpyAsync(W, t, sizeof(double2) * N, hipMemcpyDeviceToDevice, s));
        }
        const double beta = norm(W);
        res = beta / bnorm;
        if (res <= tol || it >= max_iter) break;
        axpby_abi(W, W, 0.0, 1.0 / beta, false, (size_t)N, s);
        std::fill(gv.begin(), gv.end(), cplx(0.0, 0.0));
        gv[0] = beta;
        int j = 0;
        while (j < R && it < max_iter) {
          double2* w = W + (size_t)(j + 1) * ld;
          apply_D(W + (size_t)j * ld, w);
          ++it;
          gs_dot(g, W, ld, N, j + 1, w, h1, s, nullptr);
          gs_update(g, W, ld, N, j + 1, h1, w, nullptr, 0, s, nullptr);
          gs_dot(g, W, ld, N, j + 1, w, h2, s, nullptr);
          SGN_HIP(hipMemsetAsync(dflag, 0, sizeof(int), s));
          GsFinal fin{h1, hout, nullptr, nullptr, dflag};
          gs_update(g, W, ld, N, j + 1, h2, w, &fin, 0, s, nullptr);
          int hflag = 0;
          SGN_HIP(hipMemcpyAsync(hh.data(), hout, sizeof(double2) * (j + 2), hipMemcpyDeviceToHost, s));
          SGN_HIP(hipMemcpyAsync(&hflag, dflag, sizeof(int), hipMemcpyDeviceToHost, s));
          SGN_HIP(hipStreamSynchronize(s));
          // the update kernel writes 0 in place of a non-finite norm; its flag
          // (-1) and the coefficients tell a NaN column from a lucky breakdown
          bool finite = hflag >= 0;
          for (int i = 0; i <= j + 1; ++i) finite = finite && std::isfinite(hh[i].x) && std::isfinite(hh[i].y);
          SGN_REQUIRE(finite, SGN_EINVAL, "overlap solve: non-finite value in the outer Arnoldi basis");
          const double hn = hh[j + 1].x;
          cplx* Hj = &H[(size_t)j * (R + 1)];
          for (int i = 0; i <= j; ++i) Hj[i] = cplx(hh[i].x, hh[i].y);
          Hj[j + 1] = hn;
          for (int i = 0; i < j; ++i) {  // earlier rotations
            const cplx u = Hj[i], v = Hj[i + 1];
            Hj[i] = cs[i] * u + sn[i] * v;
            Hj[i + 1] = -std::conj(sn[i]) * u + cs[i] * v;
          }
          const double r = std::hypot(std::abs(Hj[j]), hn);
          if (std::abs(Hj[j]) == 0.0) {
            cs[j] = 0.0;
            sn[j] = 1.0;
          } else {
            const cplx ph = Hj[j] / std::abs(Hj[j]);
            cs[j] = std::abs(Hj[j]) / r;
            sn[j] = ph * hn / r;
          }
          Hj[j] = cs[j] * Hj[j] + sn[j] * Hj[j + 1];
          Hj[j + 1] = 0.0;
          gv[j + 1] = -std::conj(sn[j]) * gv[j];
          gv[j] = cs[j] * gv[j];
          ++j;
          if (hn > 0.0) axpby_abi(w, w, 0.0, 1.0 / hn, false, (size_t)N, s);
          if (std::abs(gv[j]) <= tol * bnorm || hn == 0.0) break;
        }
        // x += W y with R y = g (upper triangular j x j)
        for (int i = j - 1; i >= 0; --i) {
          cplx acc = gv[i];
          for (int k = i + 1; k < j; ++k) acc -= H[(size_t)k * (R + 1) + i] * y[k];
          y[i] = acc / H[(size_t)i * (R + 1) + i];
        }
        for (int i = 0; i < j; ++i) hh[i] = make_double2(y[i].real(), y[i].imag());
        SGN_HIP(hipMemcpyAsync(hout, hh.data(), sizeof(double2) * j, hipMemcpyHostToDevice, s));
        gs_add(g, W, ld, N, j, hout, x2, s, nullptr);
        SGN_HIP(hipStreamSynchronize(s));  // hh is pageable host memory
      }
    }
    if (iters) *iters = it;
    if (rel_res) *rel_res = res;
    if (res > tol) {
      c->last_error = "overlap solve: max_iter reached before the requested tolerance";
      return SGN_ENOCONV;
    }
    return SGN_OK;
  });
}

int sgn_debug_hessenberg(const sgn_ctx* cc, int n, double* H, double* c0, double* beta) {
  sgn_ctx* c = const_cast<sgn_ctx*>(cc);
  return guarded(c, [&] {
    SGN_REQUIRE(c->Hc && n >= 0 && n <= c->ncap, SGN_EINVAL, "no Hessenberg of that size");
    SGN_HIP(hipStreamSynchronize(c->stream));
    if (H && n)
      SGN_HIP(hipMemcpy2D(H, sizeof(double2) * n, c->Hc, sizeof(double2) * c->ncap, sizeof(double2) * n, n,
                          hipMemcpyDeviceToHost));
    if (c0 && c->m) SGN_HIP(hipMemcpy(c0, c->c0, sizeof(double2) * c->m, hipMemcpyDeviceToHost));
    if (beta) SGN_HIP(hipMemcpy(beta, &c->scal[0], sizeof(double), hipMemcpyDeviceToHost));
    return SGN_OK;
  });
}

int sgn_set_precision(sgn_ctx* c, int prec) {
  return guarded(c, [&] {
    SGN_REQUIRE(prec == SGN_PREC_FP64 || prec == SGN_PREC_MIXED, SGN_EINVAL, "unknown precision");
    SGN_REQUIRE(c->sessions == 0 || prec == c->prec, SGN_ESTATE, "a serving session holds this field's precision");
    SGN_HIP(hipStreamSynchronize(c->stream));
    if (prec == c->prec) return SGN_OK;
    c->release_workspace();
    c->bw.release();
    c->prec = prec;
    c->k_hint = 0;
    c->rate_hint = 0.0;
    c->bw.k_hint = 0;
    c->bw.rate_hint = 0.0;
    if (prec == SGN_PREC_MIXED && !c->links32) {
      SGN_HIP(hipMalloc(&c->links32, sizeof(float2) * wilson_link_entries(c->lat.V)));
      wilson_links_f32(c->links, c->links32, c->lat.V, c->stream);
      SGN_HIP(hipStreamSynchronize(c->stream));
    }
    return SGN_OK;
  });
}

int sgn_get_precision(const sgn_ctx* c) { return c ? c->prec : SGN_ESTATE; }

int sgn_set_schedule(sgn_ctx* c, int k_first, double tol) {
  return guarded(c, [&] {
    SGN_REQUIRE(k_first >= 0, SGN_EINVAL, "k_first must be >= 0");
    c->k_hint = k_first;
    c->tol_hint = tol;
    c->rate_hint = 0.0;
    c->bw.k_hint = k_first;
    c->bw.tol_hint = tol;
    c->bw.rate_hint = 0.0;
    return SGN_OK;
  });
}

int sgn_set_sign_method(sgn_ctx* c, int method) {
  return guarded(c, [&] {
    SGN_REQUIRE(method == SGN_SIGN_SCHULZ || method == SGN_SIGN_ROBERTS, SGN_EINVAL, "unknown sign method");
    c->dense.method = method;
    return SGN_OK;
  });
}

int sgn_set_orthogonalization(sgn_ctx* c, int mode) {
  return guarded(c, [&] {
    SGN_REQUIRE(mode == SGN_ORTH_CGS2 || mode == SGN_ORTH_DELAYED, SGN_EINVAL, "unknown orthogonalisation mode");
    c->orth = mode;
    return SGN_OK;
  });
}

int sgn_set_block_steps(sgn_ctx* c, int sb) {
  return guarded(c, [&] {
    SGN_REQUIRE(sb >= 0 && sb <= kBlockMax, SGN_EINVAL, "block steps must be 0 (off) or 1..16");
    c->block_s = sb;
    return SGN_OK;
  });
}

int sgn_get_block_steps(const sgn_ctx* cc, int* sb, double* e_out) {
  sgn_ctx* c = const_cast<sgn_ctx*>(cc);
  return guarded(c, [&] {
    if (sb) *sb = c->block_s;
    if (e_out) *e_out = c->cheb_e;
    return SGN_OK;
  });
}

int sgn_set_tuning(sgn_ctx* c, int update_batch, int dot_cols, int update_waves) {
  return guarded(c, [&] {
    KrylovTune t;
    t.ub = update_batch;
    t.cpw = dot_cols;
    t.uw = update_waves;
    SGN_REQUIRE(krylov_tune_valid(t), SGN_EINVAL,
                "update_batch must be 4, 8 or 16, dot_cols 1, 2 or 4 and update_waves 8 or 16");
    SGN_HIP(hipStreamSynchronize(c->stream));
    c->tune = t;
    c->drop_graphs();  // they hold the previous kernel instances
    return SGN_OK;
  });
}

int sgn_set_stencil_blocks(sgn_ctx* c, int By, int Bz, int Bt) {
  return guarded(c, [&] {
    SGN_REQUIRE(wilson_blocks_valid(c->lat, By, Bz, Bt), SGN_EINVAL,
                "blocks must divide Ly, Lz, Lt with Lx*By a multiple of 32 (0,0,0: default; -1: natural order)");
    SGN_HIP(hipStreamSynchronize(c->stream));
    c->lat.blk[0] = By < 0 ? -1 : By;
    c->lat.blk[1] = By < 0 ? 0 : Bz;
    c->lat.blk[2] = By < 0 ? 0 : Bt;
    c->drop_graphs();  // captured stencil launches hold the old order
    return SGN_OK;
  });
}

int sgn_set_step_graphs(sgn_ctx* c, int steps) {
  return guarded(c, [&] {
    SGN_REQUIRE(steps == 0 || (steps >= 2 && steps <= 64), SGN_EINVAL, "steps must be 0 or 2..64");
    SGN_HIP(hipStreamSynchronize(c->stream));
    if (steps != c->graph_steps) c->drop_graphs();
    c->graph_steps = steps;
    return SGN_OK;
  });
}

int sgn_get_tuning(const sgn_ctx* c, int* update_batch, int* dot_cols, int* update_waves) {
  if (!c) return SGN_ESTATE;
  if (!update_batch || !dot_cols || !update_waves) return SGN_EINVAL;
  *update_batch = c->tune.ub;
  *dot_cols = c->tune.cpw;
  *update_waves = c->tune.uw;
  return SGN_OK;
}

int sgn_last_info(const sgn_ctx* c, sgn_info* info) {
  if (!c) return SGN_ESTATE;
  if (!info) return SGN_EINVAL;
  *info = c->info;
  return SGN_OK;
}

size_t sgn_footprint_bytes(const sgn_ctx* c, int kmax, int nrhs) {
  if (!c || kmax < 0 || nrhs < 1) return 0;
  if (nrhs > 1) {
    // sgn_apply_batched: per chunk of at most 64 sources
    const size_t vt = c->prec == SGN_PREC_MIXED ? sizeof(float2) : sizeof(double2);
    return BatchWork::bytes(c->ldq, c->m, std::max(kmax, 2), std::min(nrhs, kMaxBatch), vt) +
           sizeof(double2) * c->ldq * (size_t)std::max(c->m, 1);
  }
  const size_t ncap = (size_t)c->m + kmax + 1;
  const size_t per = sizeof(double2) * (c->ldq * (ncap + 3) + ncap * ncap + (ncap - 1) * (ncap - 1) + 4 * ncap) +
                     sizeof(double2) * c->ldq * ((ncap + 31) / 32);
  const size_t dense = 3 * sizeof(double2) * (ncap - 1) * (ncap - 1);
  return per + dense;
}

int sgn_matvec(sgn_ctx* c, const double* x, double* y) {
  return guarded(c, [&] {
    SGN_REQUIRE(x && y && x != y, SGN_EINVAL, "x and y must be distinct non-NULL buffers");
    double2 *a = nullptr, *b = nullptr;
    SGN_HIP(hipMalloc(&a, sizeof(double2) * c->ldq));
    SGN_HIP(hipMalloc(&b, sizeof(double2) * c->ldq));
    try {
      wilson_pack(c->lat, reinterpret_cast<const double2*>(x), a, c->stream);
      wilson_apply(c->lat, c->links, a, b, nullptr, nullptr, c->stream, c->prof.on ? &c->prof : nullptr);
      wilson_unpack(c->lat, b, reinterpret_cast<double2*>(y), c->stream);
      SGN_HIP(hipStreamSynchronize(c->stream));
      if (c->prof.on) c->prof.flush();
    } catch (...) {
      (void)hipFree(a);
      (void)hipFree(b);
      throw;
    }
    SGN_HIP(hipFree(a));
    SGN_HIP(hipFree(b));
    return SGN_OK;
  });
}

int sgn_matvec_noalloc(sgn_ctx* c, const double* x, double* y) {
  return guarded(c, [&] {
    SGN_REQUIRE(x && y && x != y, SGN_EINVAL, "x and y must be distinct non-NULL buffers");
    const size_t need = 2 * sizeof(double2) * c->ldq;
    SGN_REQUIRE(need <= kScratchBytes, SGN_EINVAL,
                "lattice too large for the static staging buffer (2 * 16 * ceil(12 V / 64) * 64 bytes must be "
                "<= 64 MiB, i.e. at most 174762 sites)");
    int dev = -1;
    SGN_HIP(hipGetDevice(&dev));
    SGN_REQUIRE(dev == c->device, SGN_ESTATE, "the context's device must be current");
    auto* base = static_cast<double2*>(scratch_device_ptr(dev));
    double2* a = base;
    double2* b = base + c->ldq;
    wilson_pack(c->lat, reinterpret_cast<const double2*>(x), a, c->stream);
    wilson_apply(c->lat, c->links, a, b, nullptr, nullptr, c->stream, nullptr);
    wilson_unpack(c->lat, b, reinterpret_cast<double2*>(y), c->stream);
    SGN_HIP(hipStreamSynchronize(c->stream));
    return SGN_OK;
  });
}

int sgn_dense_sign(sgn_ctx* c, int n, const double* A, double* F, int* iters) {
  return guarded(c, [&] {
    SGN_REQUIRE(n >= 1 && A && F, SGN_EINVAL, "need n >= 1 and non-NULL A, F");
    c->prof.stream = c->stream;
    const int it = dense_sign(c->dense, n, reinterpret_cast<const double2*>(A), n, reinterpret_cast<double2*>(F), n,
                              c->stream, c->prof.on ? &c->prof : nullptr);
    SGN_HIP(hipStreamSynchronize(c->stream));
    if (c->prof.on) c->prof.flush();
    if (iters) *iters = it;
    return SGN_OK;
  });
}

int sgn_zgemm(sgn_ctx* c, int M, int N, int K, const double* A, int lda, const double* B, int ldb, double* C,
              int ldc) {
  return guarded(c, [&] {
    SGN_REQUIRE(M >= 0 && N >= 0 && K >= 0, SGN_EINVAL, "sizes must be >= 0");
    SGN_REQUIRE(lda >= std::max(M, 1) && ldb >= std::max(K, 1) && ldc >= std::max(M, 1), SGN_EINVAL,
                "leading dimensions too small");
    if (M == 0 || N == 0) return SGN_OK;
    SGN_REQUIRE(C && ((A && B) || K == 0), SGN_EINVAL, "NULL matrix");
    if (K == 0) {
      for (int j = 0; j < N; ++j) dev_zero(reinterpret_cast<double2*>(C) + (size_t)j * ldc, (size_t)M, c->stream);
    } else {
      zgemm(M, N, K, 1.0, reinterpret_cast<const double2*>(A), lda, 0, reinterpret_cast<const double2*>(B), ldb, 0,
            reinterpret_cast<double2*>(C), ldc, 0, 1, c->stream);
    }
    SGN_HIP(hipStreamSynchronize(c->stream));
    return SGN_OK;
  });
}

int sgn_set_profiling(sgn_ctx* c, int on) {
  return guarded(c, [&] {
    c->prof.stream = c->stream;
    if (!on) c->prof.flush();
    c->prof.on = on != 0;
    return SGN_OK;
  });
}

int sgn_profile_read(const sgn_ctx* cc, sgn_kstat* out, int max) {
  sgn_ctx* c = const_cast<sgn_ctx*>(cc);
  return guarded(c, [&] {
    c->prof.flush();
    int cnt = 0;
    for (int k = 0; k < K_NCLASS && cnt < max; ++k) {
      if (!out) break;
      sgn_kstat& o = out[cnt++];
      std::memset(&o, 0, sizeof(o));
      std::strncpy(o.name, kclass_name(k), sizeof(o.name) - 1);
      o.launches = c->prof.launches[k];
      o.ms = c->prof.ms[k];
      o.bytes = c->prof.bytes[k];
      o.flops = c->prof.flops[k];
    }
    return cnt;
  });
}

int sgn_profile_reset(sgn_ctx* c) {
  return guarded(c, [&] {
    c->prof.flush();
    c->prof.reset();
    return SGN_OK;
  });
}

}  // extern "C"
