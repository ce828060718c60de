// One-reduction modified Arnoldi step (krylov.hip): argument block and workspace.
#pragma once

#include <algorithm>

#include "internal.h"

// per-slot step scalars (doubles), kScStride apart
enum {
  kScC = 0,      // u^dag u
  kScRho,        // |u| after re-orthogonalisation (0 on breakdown)
  kScInv,        // 1 / rho (0 on breakdown)
  kScGamRe,      // gam = q_J^dag z
  kScGamIm,
  kScGrRe,       // gam / rho
  kScGrIm,
  kScScale,      // |z| / rho: reference size of the next candidate
  kScRef,        // reference size for the breakdown test of an even step (odd: kScRef + 1)
  kScRefOdd,
  kScRawC,       // raw sums of the dot pass: u^dag u, u^dag z (re, im), |z|^2 (4 slots)
  kScStride = 16
};

// Launch shape of the dot and update passes.  Every choice of ub and cpw
// forms every sum in the same order, so results do not depend on them; only
// the time does.
//   ub:  update pass, column loads per lane issued before their arithmetic (4, 8, 16)
//   cpw: dot pass, columns per wavefront (1, 2, 4): fewer columns per
//        wavefront means more workgroups, shorter chains of dependent loads,
//        and more re-reads of u and z from cache
//   uw:  update pass, wavefronts per 64-row workgroup (8, 16).  Unlike ub and
//        cpw this changes which columns each wavefront sums, so results
//        differ at the rounding level between its values (every path of a
//        context uses the same value, so they stay bitwise consistent).
struct KrylovTune {
  int ub = 8;
  int cpw = 4;
  int uw = 8;
};
bool krylov_tune_valid(const KrylovTune& t);

struct KrylovArgs {
  int N = 0;
  size_t ldq = 0;
  int m = 0;                    // Schur columns (FP64, shared by all slots)
  const double2* S = nullptr;   // ldq x m
  // launch z (blockIdx.z < nb) works on slot act[z], whose step index is
  // jv[z]: its basis has J = m + jv[z] finished columns
  int nb = 1;
  int act[kMaxBatch] = {};
  int jv[kMaxBatch] = {};
  // replayable launches: the step index of every launch slot is *jdev + joff,
  // read on the device; jv[] then only sizes the grids (an upper bound)
  const int* jdev = nullptr;
  int joff = 0;
  // Krylov columns: column c >= m of slot r at V + r*vstride + (c-m)*ldq (element type VT)
  void* V = nullptr;
  size_t vstride = 0;
  // FP64 candidate u (read) and next candidate (written; may equal u), per
  // slot at ustride
  double2* u = nullptr;
  double2* unext = nullptr;
  size_t ustride = 0;
  // stencil result z (VT, read) and the VT copy of the next candidate (written; nullable)
  const void* z = nullptr;
  void* ulonext = nullptr;
  size_t zstride = 0;
  // composite Hessenberg per slot
  double2* H = nullptr;
  int ldh = 0;
  size_t hstride = 0;
  double2* c0 = nullptr;  // S^dag x per slot (m entries at c0stride)
  int c0stride = 0;
  double* beta = nullptr;  // |x_perp| per slot (written at j = 0)
  int* flag = nullptr;     // breakdown record per slot: k_invariant + 1, or -1 for non-finite values
  // the Krylov space counts as invariant when the new candidate's norm after
  // orthogonalisation is below brk_tol times its reference size: about the
  // rounding level of the stored basis (FP64: 1e-12; FP32 columns: 1e-6)
  double brk_tol = 1e-12;
  KrylovTune tune;  // host side only (selects the kernel instance)
  // filled by krylov_bind from the workspace
  double2 *Pa = nullptr, *Pb = nullptr;
  double* Pcd = nullptr;
  int ldp = 0;
  size_t pstride = 0, cdstride = 0;
  double2 *a = nullptr, *b = nullptr;
  size_t abstride = 0;
  double* sc = nullptr;
  int nrt_dot = 0;

  // host helpers
  void single(int j) {  // one right-hand side in slot 0
    nb = 1;
    act[0] = 0;
    jv[0] = j;
  }
  int jmax() const {
    int x = 0;
    for (int z = 0; z < nb; ++z) x = jv[z] > x ? jv[z] : x;
    return x;
  }
};

// partial sums of the dot pass [slot][row tile][column], the reduced
// coefficients a, b [slot][column] and the step scalars [slot][kScStride]
struct KrylovWork {
  int nrt_dot = 0, ncol_cap = 0, nslots = 0;
  int ldp = 0;
  size_t pstride = 0, cdstride = 0, abstride = 0;
  double2 *Pa = nullptr, *Pb = nullptr;
  double* Pcd = nullptr;
  double2 *a = nullptr, *b = nullptr;
  double* sc = nullptr;
};

void krylov_alloc(KrylovWork& w, int N, size_t ldq, int ncol_cap, int nslots);
void krylov_free(KrylovWork& w);
void krylov_bind(const KrylovWork& w, KrylovArgs& A);

// a = Q_J^dag u, b = Q_J^dag z (if with_z), raw scalars; per launch slot
template <typename VT>
void krylov_dot(const KrylovWork& w, const KrylovArgs& A, bool with_z, hipStream_t s, Profiler* prof);
// v_J, next candidate, Hessenberg column J and re-orthogonalisation of column J-1
template <typename VT>
void krylov_update(const KrylovWork& w, const KrylovArgs& A, hipStream_t s, Profiler* prof);
// *p = v, or *p += v (stream-ordered; for the device step index of replayed steps)
void krylov_set_index(int* p, int v, bool add, hipStream_t s);
// y_r = Q_r coef_r over ncol columns (the same ncol for every launch slot)
template <typename VT>
void krylov_combine(const KrylovWork& w, const KrylovArgs& A, const double2* coef, int cstride, double2* y,
                    size_t ystride, int ncol, hipStream_t s, Profiler* prof);
// dst_z = H_r[:n,:n] (dense n x n at dstride, z = launch slot, r = act[z]) with
// column n-1 += a_r when with_a
void krylov_patch(const KrylovWork& w, const KrylovArgs& A, int n, double2* dst, size_t dstride, bool with_a,
                  hipStream_t s);
