// psd_kernels.hpp -- __global__ kernels of the PSD solver (gfx950).
// Every kernel reads its unit of work from a task table and its problem from
// an instance table, so one launch can serve one large instance or a batch
// of instances of different sizes.  Solver kernels return at once when their
// instance is finished (SolveState::done), which lets a captured graph of
// several iterations be replayed past convergence at negligible cost.
#pragma once
#include "psd_common.hpp"
#include "psd_fft.hpp"
#include "psd_stencil.hpp"

namespace psd {

struct Task2 {  // residual / line-search / col tiles
  int inst, a, b, c, slot, pad0, pad1, pad2;
};

// ---------------------------------------------------------------------------
// supported line lengths
// ---------------------------------------------------------------------------
#define PSD_FOR_EACH_N(X) X(16) X(32) X(48) X(64) X(96) X(128) X(192) X(256) X(384) X(512) X(1024)
// lengths of the 3D grids (y-axis column passes exist in 3D only)
#define PSD_FOR_EACH_N3(X) X(32) X(48) X(64) X(96) X(128) X(192) X(256)

// Lines per block of the row passes (LDS layout of the row transform): the
// largest power of two whose lines fit in about PSD_ROW_BYTES of LDS scaled
// by 2^(SEL-1); the autotuner picks SEL in 0..PSD_ROW_SELS-1 per handle.
#ifndef PSD_ROW_BYTES
#define PSD_ROW_BYTES 32768
#endif
constexpr int PSD_ROW_SELS = 3;
template <typename T, int N, int SEL = 1>
constexpr int row_lines() {
  int nl = ((PSD_ROW_BYTES << SEL) / 2) / (fft_ls(N) * (int)sizeof(cx<T>));  // plus N twiddles
  int p = 1;
  while (p * 2 <= nl && p < 32) p *= 2;
  return p;
}
// columns per block of a column pass: 128-byte segments where the LDS
// footprint NF*W*fft_ls(N) complex plus N twiddles and N doubles of the
// symbol (fused pass) stays within 64 KB; a power of two, so that a thread
// keeps one column
#ifndef PSD_COL_BYTES
#define PSD_COL_BYTES 128
#endif
template <typename T, int N, int NF>
constexpr int col_width() {
  if (NF == 1 && col_four_step<T, N>()) return four_step_width<N>();
  int w = PSD_COL_BYTES / (int)sizeof(cx<T>);
  // 64 KB per block: W columns per field, twiddles, and (fused pass) the symbol
  const int cap = (65536 - N * (int)sizeof(cx<T>) - N * 8) / (NF * fft_ls(N) * (int)sizeof(cx<T>));
  while (w > cap && w > 1) w /= 2;
  return w;
}

// ===========================================================================
// residual (+ fused update)
// ===========================================================================
template <typename TD, typename TR, int ORDER, bool UPD>
__global__ __launch_bounds__(PSD_NT) void k_res2d(const Inst* __restrict__ insts,
                                                  const Task2* __restrict__ tasks) {
  extern __shared__ double smem[];
  const Task2 t = tasks[blockIdx.x];
  const Inst& I = insts[t.inst];
  if (I.st->done) return;
  double acc[2] = {0.0, 0.0};
  res2d_tile<TD, TR, ORDER, UPD>(I, t.a, t.b, smem, acc);
  block_reduce<2, 1>(acc, smem + R2_LDS);
  if (threadIdx.x == 0) {
    I.part_res[2 * t.slot] = acc[0];
    I.part_res[2 * t.slot + 1] = acc[1];
  }
}

// Register budget of the 3D residual: two cells per thread need up to 232
// VGPRs (general p), so 2 waves per SIMD; at 3 waves the p = 4 mixed kernel
// fits but measured slower (125 against 117 us at 256^3) and the general-p
// and FP64 ones spill.
constexpr int RES3D_WAVES = 2;
template <typename TD, typename TR, bool UPD, int PK, int TX>
__global__ __launch_bounds__(PSD_NT) __attribute__((amdgpu_waves_per_eu(RES3D_WAVES))) void k_res3d(const Inst* __restrict__ insts,
                                                  const Task2* __restrict__ tasks) {
  extern __shared__ double smem[];
  const Task2 t = tasks[blockIdx.x];
  const Inst& I = insts[t.inst];
  if (I.st->done) return;
  double acc[2] = {0.0, 0.0};
  res3d_tile<TD, TR, UPD, false, PK, TX>(I, t.a, t.b, t.c, smem, acc);
  block_reduce<2, 1>(acc, smem + R3Shape<TX>::LDS);
  if (threadIdx.x == 0) {
    I.part_res[2 * t.slot] = acc[0];
    I.part_res[2 * t.slot + 1] = acc[1];
  }
}

// 3D sixth-order residual (brick tiles, res3d6_tile)
template <typename TD, typename TR, bool UPD>
__global__ __launch_bounds__(PSD_NT) void k_res3d6(const Inst* __restrict__ insts,
                                                   const Task2* __restrict__ tasks) {
  extern __shared__ double smem[];
  const Task2 t = tasks[blockIdx.x];
  const Inst& I = insts[t.inst];
  if (I.st->done) return;
  double acc[2] = {0.0, 0.0};
  res3d6_tile<TD, TR, UPD>(I, t.a, t.b, t.c, smem, acc);
  block_reduce<2, 1>(acc, smem + B6_LDS);
  if (threadIdx.x == 0) {
    I.part_res[2 * t.slot] = acc[0];
    I.part_res[2 * t.slot + 1] = acc[1];
  }
}

// One block per instance: reduce residual partials, count the update,
// decide convergence, record history.
__global__ __launch_bounds__(PSD_FIN_NT) void k_res_finalize(const Inst* __restrict__ insts, int upd) {
  __shared__ double scratch[2 * PSD_FIN_NT / PSD_WAVE];
  const Inst& I = insts[blockIdx.x];
  SolveState* st = I.st;
  const int done = st->done;   // loaded together with the partials
  double acc[2] = {0.0, 0.0};
  flat_reduce<2, 1, PSD_FIN_NT>(I.part_res, I.nblk_res, acc, scratch);
  if (done) return;
  if (threadIdx.x == 0) {
    const double rinf = acc[0];
    const double rl2 = sqrt(I.hd * acc[1]);
    st->rinf = rinf;
    st->rl2 = rl2;
    if (upd) {
      st->iter += 1;
      if (I.hist && st->iter <= I.hist_cap) {
        double* hrec = I.hist + 4 * (st->iter - 1);
        hrec[0] = st->alpha; hrec[1] = rinf; hrec[2] = rl2; hrec[3] = st->dE;
      }
    }
    if (!isfinite(acc[1])) { st->status = -4; st->done = 1; }
    else if (rinf <= I.tol) { st->status = 0; st->done = 1; }
    else if (st->iter >= I.max_iter) { st->status = 1; st->done = 1; }
  }
}

// ===========================================================================
// line search
// ===========================================================================
template <typename TD, int MODE>
__global__ __launch_bounds__(PSD_NT) void k_ls2d(const Inst* __restrict__ insts,
                                                 const Task2* __restrict__ tasks) {
  extern __shared__ double smem[];
  const Task2 t = tasks[blockIdx.x];
  const Inst& I = insts[t.inst];
  if (I.st->done || (MODE == 2 && I.st->ls_phase == 2)) return;
  double acc[8] = {0, 0, 0, 0, 0, 0, 0, 0};
  ls2d_wave_tile<TD, MODE>(I, t.a, t.b, acc);
  block_reduce<8, 0>(acc, smem);
  if (threadIdx.x == 0)
    for (int k = 0; k < 8; ++k) I.part_ls[8 * t.slot + k] = acc[k];
}

template <typename TD, int MODE, int TX>
__global__ __launch_bounds__(PSD_NT) void k_ls3d(const Inst* __restrict__ insts,
                                                 const Task2* __restrict__ tasks) {
  extern __shared__ double smem[];
  const Task2 t = tasks[blockIdx.x];
  const Inst& I = insts[t.inst];
  if (I.st->done || (MODE == 2 && I.st->ls_phase == 2)) return;
  double acc[8] = {0, 0, 0, 0, 0, 0, 0, 0};
  ls3d_tile<TD, MODE, TX>(I, t.a, t.b, t.c, smem, acc);
  block_reduce<8, 0>(acc, smem + L3Shape<TX>::LDS);
  if (threadIdx.x == 0)
    for (int k = 0; k < 8; ++k) I.part_ls[8 * t.slot + k] = acc[k];
}

// q(x) = c0 + c1 x + ... + cD x^D and q'(x) by Horner's rule
template <int D>
__device__ __forceinline__ void poly_eval(const double* c, double x, double& q, double& dq) {
  q = c[D];
  dq = 0.0;
#pragma unroll
  for (int k = D - 1; k >= 0; --k) {
    dq = dq * x + q;
    q = q * x + c[k];
  }
}

// Root of the strictly increasing polynomial q of degree D: the cubic (p = 4)
// or quintic (p = 6) of Sec. 6.1.  Rule: x = -c0/c1, double until q > 0, then
// Newton from that point with bisection whenever a step leaves the bracket;
// stop when |q| <= 1e-16 (|c0| + c1 x) or |dx| <= 1e-15 x.
template <int D>
__device__ double poly_root(const double* c) {
  double lo = 0.0, hi = INFINITY, x = -c[0] / c[1], q = 0.0, dq = 0.0;
  for (int it = 0; it < 200; ++it) {
    poly_eval<D>(c, x, q, dq);
    if (q > 0.0) { hi = x; break; }
    if (q == 0.0) return x;
    lo = x;
    x *= 2.0;
  }
  for (int it = 0; it < 100; ++it) {
    if (fabs(q) <= 1e-16 * (fabs(c[0]) + c[1] * x)) break;
    double xn = x - q / dq;
    if (!(xn > lo && xn < hi)) xn = 0.5 * (lo + hi);
    if (fabs(xn - x) <= 1e-15 * x) { x = xn; break; }
    x = xn;
    poly_eval<D>(c, x, q, dq);
    if (q > 0.0) hi = x;
    else if (q < 0.0) lo = x;
    else break;
  }
  return x;
}

// Reduce line-search and spectral partials; mode 0: cubic (p = 4) -> alpha;
// mode 3: quintic (p = 6) -> alpha; mode 1: general p, first pass at
// alpha = 0 -> start the root search; mode 2: general p, one step of the
// root search after an evaluation of (q, q') at st->x.
//
// General-p root search (q strictly increasing, Sec. 6.1): safeguarded Newton
// from x0 = -q(0)/q'(0).  Each evaluation narrows the bracket [lo, hi] by the
// sign of q; a Newton step that leaves the bracket is replaced by bisection
// (doubling while no upper end is known).  It stops at |q| <= 1e-16 (|q(0)| +
// q'(0) x), or takes the Newton iterate without evaluating it once the
// Newton step is below 1e-8 x: with quadratic convergence its error is then
// at the level of rounding.  After max_evals evaluations it takes its best
// estimate and counts the search in st->ls_trunc (graph-captured iterations
// run a fixed number of evaluation passes).
__global__ __launch_bounds__(PSD_FIN_NT) void k_ls_finalize(const Inst* __restrict__ insts, int mode,
                                                            int max_evals) {
  __shared__ double scratch[10 * PSD_FIN_NT / PSD_WAVE];
  const Inst& I = insts[blockIdx.x];
  SolveState* st = I.st;
  // Mode 2: the passes captured after the root search has finished are the
  // common case, so the state is read first and the partials only if needed.
  // Modes 0, 1, 3 (the pass almost always has work): the state's flag is
  // loaded with the partials and tested only after their reduction, so that
  // both arrive in one memory round trip (the empty asm statement below keeps
  // the compiler from comparing the flag, and so waiting for its load, before
  // the partials' loads are issued).
  int skip = 0;
  if (mode == 2) {
    if (st->done || st->ls_phase == 2) return;
  } else {
    skip = st->done;
  }
  double acc[10] = {0, 0, 0, 0, 0, 0, 0, 0, 0, 0};
  {
    double a8[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    double a2[2] = {0.0, 0.0};
    flat_reduce2<8, 2, PSD_FIN_NT>(I.part_ls, I.nblk_ls, I.part_sp, mode != 2 ? I.nblk_sp : 0, a8, a2,
                                   scratch);
#pragma unroll
    for (int k = 0; k < 8; ++k) acc[k] = a8[k];
    acc[8] = a2[0];
    acc[9] = a2[1];
  }
  __asm__ volatile("" : "+v"(skip));
  if (skip) return;
  if (I.order == 6 && mode != 2) {
    // means of d, e1, e2 (FP32 round-off of the inverse transform leaves a
    // tiny mean that the preconditioner never corrects); the update removes them
    double ms[3] = {0.0, 0.0, 0.0};
    gather_parts<3, 0>(I.part_c2r, I.nblk_c2r, ms);
    block_reduce<3, 0, PSD_FIN_NT>(ms, scratch);
    if (threadIdx.x == 0) {
      for (int q = 0; q < 3; ++q) st->mean[q] = ms[q] * I.inv_ntot;
      // sum (d - dbar)^2 = sum d^2 - N dbar^2
      const double corr = (double)I.ncell * st->mean[0] * st->mean[0];
      if (mode == 0) acc[4] -= corr; else if (mode == 3) acc[5] -= corr; else acc[2] -= corr;
    }
  }
  if (threadIdx.x != 0) return;
  const double s = I.s, se2 = I.se2;
  if (mode == 0) {
    const double S2 = acc[0], S3 = acc[1], S4 = acc[2], S5 = acc[3], P2 = acc[4], P4 = acc[5];
    const double lin = (I.order == 4) ? P2 : s * I.lam * P2 + acc[9];
    double c[4];
    c[0] = -acc[8];
    c[1] = lin + s * (S2 + 2.0 * S3) + se2 * P4;
    c[2] = 3.0 * s * S4;
    c[3] = s * S5;
    for (int k = 0; k < 4; ++k) st->c[k] = c[k];
    st->c[4] = st->c[5] = 0.0;
    if (!(c[0] < 0.0) || !(c[1] > 0.0)) {
      st->status = -5; st->done = 1; st->alpha = 0.0;
      return;
    }
    const double a = poly_root<3>(c);
    st->alpha = a;
    st->dE = I.hd * a * (c[0] + a * (c[1] / 2.0 + a * (c[2] / 3.0 + a * c[3] / 4.0)));
    st->ls_phase = 2;
    return;
  }
  if (mode == 3) {
    // p = 6: q(x) = c0 + c1 x + ... + c5 x^5 with c0 = -(r, d),
    // c1 = P2 + s t1 + s eps^2 P4 (order 6: s lam P2 + (T_h d, d) in place of P2),
    // c_k = s t_k (k >= 2)
    const double P2 = acc[5], P4 = acc[6];
    const double lin = (I.order == 4) ? P2 : s * I.lam * P2 + acc[9];
    double c[6];
    c[0] = -acc[8];
    c[1] = lin + s * acc[0] + se2 * P4;
    for (int k = 2; k <= 5; ++k) c[k] = s * acc[k - 1];
    for (int k = 0; k < 6; ++k) st->c[k] = c[k];
    if (!(c[0] < 0.0) || !(c[1] > 0.0)) {
      st->status = -5; st->done = 1; st->alpha = 0.0;
      return;
    }
    const double a = poly_root<5>(c);
    st->alpha = a;
    double e = 0.0;   // integral of q from 0 to a
    for (int k = 5; k >= 0; --k) e = e * a + c[k] / (double)(k + 1);
    st->dE = I.hd * a * e;
    st->ls_phase = 2;
    return;
  }
  if (mode == 1) {
    const double NL = acc[0], dNL = acc[1], P2 = acc[2], P4 = acc[3];
    const double lin = ((I.order == 4) ? P2 : s * I.lam * P2 + acc[9]) + se2 * P4;
    const double q0 = -acc[8];
    const double dq0 = lin + s * dNL;
    st->c[0] = q0; st->c[1] = dq0; st->lin = lin; st->nl0 = NL;
    st->dE = 0.0;
    if (!(q0 < 0.0) || !(dq0 > 0.0)) {
      st->status = -5; st->done = 1; st->alpha = 0.0; st->ls_phase = 2;
      return;
    }
    st->lo = 0.0; st->hi = INFINITY; st->x = -q0 / dq0;
    st->ls_phase = 1; st->ls_evals = 0; st->newton_steps = 0;
    return;
  }
  // mode 2: evaluation at x finished
  const double x = st->x;
  const double q = st->c[0] + x * st->lin + s * (acc[0] - st->nl0);
  const double dq = st->lin + s * acc[1];
  const double c0 = st->c[0], c1 = st->c[1];
  st->ls_evals += 1;
  if (q > 0.0) st->hi = x;
  else if (q < 0.0) st->lo = x;
  else { st->alpha = x; st->ls_phase = 2; return; }
  if (fabs(q) <= 1e-16 * (fabs(c0) + c1 * x)) { st->alpha = x; st->ls_phase = 2; return; }
  double xn = x - q / dq;
  const bool newton = dq > 0.0 && xn > st->lo && xn < st->hi;
  if (!newton) xn = isfinite(st->hi) ? 0.5 * (st->lo + st->hi) : 2.0 * x;
  else st->newton_steps += 1;
  if (newton && fabs(xn - x) <= 1e-8 * x) { st->alpha = xn; st->ls_phase = 2; return; }
  if (st->ls_evals >= max_evals) {
    st->alpha = newton ? xn : x;
    st->ls_phase = 2;
    st->ls_trunc += 1;
    return;
  }
  st->x = xn;
}

// ===========================================================================
// FFT passes
// ===========================================================================
enum FieldSet { FS_RES = 0, FS_DIR = 1, FS_TMP = 2 };

template <typename T>
__device__ __forceinline__ RowArgs<T> row_args(const Inst& I, int fs, cx<T>* spec, int nf) {
  RowArgs<T> A;
  A.spec = spec;
  A.nspec = sizeof(T) == 8 ? I.nspec64 : I.nspec32;
  A.nyq = sizeof(T) == 8 ? I.nyq64 : I.nyq32;
  A.ncp = sizeof(T) == 8 ? I.ncp64 : I.ncp32;
  A.rpf = I.ncell / I.n;
  A.nrows = A.rpf * nf;
  A.rin0 = A.rin1 = nullptr;
  A.rout0 = A.rout1 = A.rout2 = nullptr;
  if (fs == FS_RES) { A.rin0 = I.r; A.rin1 = I.r1; }
  else if (fs == FS_DIR) { A.rout0 = I.d; A.rout1 = I.e1; A.rout2 = I.e2; }
  else { A.rin0 = I.tmp; A.rout0 = I.tmp; }  // FP64 scratch field
  return A;
}

// row pass kernels: task.a = first global row (over fields), task.b = field
// set, task.c = number of fields.  One kernel per row length N: every block
// of a launch works on instances with n = N.
template <typename T, typename TIO, bool FWD, int N, int SEL>
__device__ __forceinline__ void rows_body(const Inst& I, const Task2& t, double* smem, int solver) {
  cx<T>* buf = (cx<T>*)smem;
  const cx<T>* tw = (const cx<T>*)(sizeof(T) == 8 ? I.tw64 : I.tw32);
  RowArgs<T> A = row_args<T>(I, t.b, (cx<T>*)I.spec, t.c);
  double fsum[3] = {0.0, 0.0, 0.0};
  if (FWD) r2c_rows<T, TIO, N, row_lines<T, N, SEL>()>(A, t.a, buf, tw);
  else c2r_rows<T, TIO, N, row_lines<T, N, SEL>()>(A, t.a, buf, tw, fsum);
  if (!FWD && solver && I.order == 6) {   // field sums of the solver's inverse transform
    __syncthreads();
    block_reduce<3, 0>(fsum, smem);
    if (threadIdx.x == 0)
      for (int q = 0; q < 3; ++q) I.part_c2r[3 * t.slot + q] = fsum[q];
  }
}

template <typename T, typename TIO, bool FWD, int N, int SEL>
__global__ __launch_bounds__(PSD_NT) void k_rows(const Inst* __restrict__ insts,
                                                 const Task2* __restrict__ tasks, int solver) {
  extern __shared__ double smem[];
  const Task2 t = tasks[blockIdx.x];
  const Inst& I = insts[t.inst];
  if (solver && I.st->done) return;
  rows_body<T, TIO, FWD, N, SEL>(I, t, smem, solver);
}

// Batches of several grid sizes: one launch, the length chosen per block.
template <typename T, typename TIO, bool FWD, int SEL>
__global__ __launch_bounds__(PSD_NT) void k_rows_any(const Inst* __restrict__ insts,
                                                     const Task2* __restrict__ tasks, int solver) {
  extern __shared__ double smem[];
  const Task2 t = tasks[blockIdx.x];
  const Inst& I = insts[t.inst];
  if (solver && I.st->done) return;
  switch (I.n) {
#define PSD_C(NN) case NN: rows_body<T, TIO, FWD, NN, SEL>(I, t, smem, solver); break;
    PSD_FOR_EACH_N(PSD_C)
#undef PSD_C
    default: break;
  }
}

// y-axis column pass (3D): lines along y of length N.  Plain block
// (task.c = 0): columns kx = task.b .. (kx < N/2) of plane z = task.a, lines
// at stride ncp.  Nyquist block (task.c = 1): the contiguous kx = N/2 lines of
// planes task.a, task.a + 1, ... in the Nyquist plane.
template <typename T, int NF, int DIR, int N>
__device__ __forceinline__ void cols_body(const Inst& I, const Task2& t, double* smem) {
  constexpr int W = col_width<T, N, NF>();
  cx<T>* buf = (cx<T>*)smem;
  const cx<T>* tw = (const cx<T>*)(sizeof(T) == 8 ? I.tw64 : I.tw32);
  const long long ncp = sizeof(T) == 8 ? I.ncp64 : I.ncp32;
  const long long fstride = sizeof(T) == 8 ? I.nspec64 : I.nspec32;
  const long long nyq = sizeof(T) == 8 ? I.nyq64 : I.nyq32;
  ColSet cs;
  if (t.c == 0) {
    cs.cbase = (long long)t.a * N * ncp + t.b;
    cs.cstride = 1;
    cs.lstride = ncp;
    cs.ncols = min(W, N / 2 - t.b);
  } else {
    cs.cbase = nyq + (long long)t.a * N;
    cs.cstride = N;
    cs.lstride = 1;
    cs.ncols = min(W, N - t.a);
  }
  col_pass<T, N, W, NF, DIR>((cx<T>*)I.spec, cs, fstride, buf, tw);
}

template <typename T, int NF, int DIR, int N>
__global__ __launch_bounds__(PSD_NT) void k_cols(const Inst* __restrict__ insts,
                                                 const Task2* __restrict__ tasks, int solver) {
  extern __shared__ double smem[];
  const Task2 t = tasks[blockIdx.x];
  const Inst& I = insts[t.inst];
  if (solver && I.st->done) return;
  cols_body<T, NF, DIR, N>(I, t, smem);
}

template <typename T, int NF, int DIR>
__global__ __launch_bounds__(PSD_NT) void k_cols_any(const Inst* __restrict__ insts,
                                                     const Task2* __restrict__ tasks, int solver) {
  extern __shared__ double smem[];
  const Task2 t = tasks[blockIdx.x];
  const Inst& I = insts[t.inst];
  if (solver && I.st->done) return;
  switch (I.n) {
#define PSD_C(NN) case NN: cols_body<T, NF, DIR, NN>(I, t, smem); break;
    PSD_FOR_EACH_N3(PSD_C)
#undef PSD_C
    default: break;
  }
}

// Spectral operators applied between the forward and inverse transform of
// the last axis.  k indices: kx = column index mod nc, ky, kz.
//   OP_PRECOND4: d^ = r^ / sigma / Ntot, sigma = 1 + s K + s eps^2 K^2
//                (order-4 preconditioner, Sec. 5.3); partial: sum w |r^|^2/sigma/Ntot
//   OP_PRECOND6: rho^ = r2^ + r1^/K, d^ = rho^/sigma6, e1^ = r1^/K, e2^ = d^/K,
//                sigma6 = s lam + s K + s eps^2 K^2 + 1/K (Sec. 5.4), k = 0 -> 0;
//                partials: sum w |rho^|^2/sigma6/Ntot, sum w |d^|^2/K/Ntot
//   OP_POISSON:  z^ -> z^/K/Ntot (T_h = -Delta_h^{-1}), partial sum w |z^|^2/K/Ntot
// K = S[kx] + S[ky] (+ S[kz]) is the symbol of -Delta_h (appendix).
//   OP_PRECOND6S: one field, z^ = r^/sigma6/Ntot, k = 0 -> 0 (sixth-order
//                adjoint); partial sum w |r^|^2/sigma6/Ntot
enum SpecOp { OP_PRECOND4 = 0, OP_PRECOND6 = 1, OP_POISSON = 2, OP_PRECOND6S = 3 };

// Last-axis pass: lines of length N along the last axis.  Plain block
// (task.c = 0): columns kx = task.b .. (kx < N/2) of row ky = task.a (3D;
// 2D: task.a = 0), lines at stride ncp (2D) or N*ncp (3D).  Nyquist block
// (task.c = 1), kx = N/2: 3D, rows ky = task.a, task.a + 1, ... of the
// Nyquist plane (lines at stride N); 2D, the one contiguous Nyquist line.
template <typename T, int N, int W>
__device__ __forceinline__ ColSet fused_cols(const Inst& I, const Task2& t) {
  const int dim = I.dim;
  const long long ncp = sizeof(T) == 8 ? I.ncp64 : I.ncp32;
  ColSet cs;
  if (t.c == 0) {
    cs.cbase = (long long)t.a * ncp + t.b;
    cs.cstride = 1;
    cs.lstride = (dim == 2) ? ncp : (long long)N * ncp;
    cs.ncols = min(W, N / 2 - t.b);
  } else {
    cs.cbase = (sizeof(T) == 8 ? I.nyq64 : I.nyq32) + t.a;
    cs.cstride = 1;
    cs.lstride = (dim == 2) ? 1 : N;
    cs.ncols = (dim == 2) ? 1 : min(W, N - t.a);
  }
  return cs;
}

// One-field operators on one spectral value X at symbol K (wgt_inv = w/Ntot).
template <typename T, int OP>
__device__ __forceinline__ cx<T> spec_one(cx<T> X, double K, double s, double se2, double inv,
                                          double wgt_inv, double& acc0, double slam = 0.0) {
  static_assert(OP == OP_PRECOND4 || OP == OP_POISSON || OP == OP_PRECOND6S, "one-field operators");
  const double x2 = (double)X.x * X.x + (double)X.y * X.y;
  if (OP == OP_PRECOND4) {
    const double rs = rcp_pos(1.0 + s * K + se2 * K * K);   // 1 / sigma
    acc0 += wgt_inv * x2 * rs;
    return scale(X, (T)(inv * rs));
  } else if (OP == OP_PRECOND6S) {
    if (!(K > 0.0)) return mk(T(0), T(0));
    const double rs = 1.0 / (slam + s * K + se2 * K * K + 1.0 / K);
    acc0 += wgt_inv * x2 * rs;
    return scale(X, (T)(inv * rs));
  } else {
    if (!(K > 0.0)) return mk(T(0), T(0));
    acc0 += wgt_inv * x2 / K;
    return scale(X, (T)(inv / K));
  }
}

template <typename T, int N, int W, int OP>
__device__ __forceinline__ void fused_col(const Inst& I, const Task2& t, cx<T>* buf, double (&acc)[2]) {
  constexpr int NFI = (OP == OP_PRECOND6) ? 2 : 1;
  constexpr int NFO = (OP == OP_PRECOND6) ? 3 : 1;
  constexpr int LS = fft_ls(N);
  static_assert(PSD_NT % W == 0, "a thread keeps one column");
  const cx<T>* tw = (const cx<T>*)(sizeof(T) == 8 ? I.tw64 : I.tw32);
  const int dim = I.dim;
  const long long fstride = sizeof(T) == 8 ? I.nspec64 : I.nspec32;
  cx<T>* base = (cx<T>*)I.spec;
  const bool nyq = t.c != 0;
  const ColSet cs = fused_cols<T, N, W>(I, t);
  constexpr int NLMAX = (NFI > NFO ? NFI : NFO) * W;
  cx<T>* twl = buf + NLMAX * LS;
  // the symbol S(k) of the last axis, staged with the twiddles
  double* Sl = (double*)(twl + N);
  TableStage<cx<T>, N> tws;
  TableStage<double, N> sst;
  col_load<T, N, W, NFI>(base, cs, fstride, buf, [&] {
    tws.load(tw);
    sst.load(I.S);
    tws.store(twl);
    sst.store(Sl);
  });
  __syncthreads();
  lds_fft<T, N, NFI * W, LS, -1>(buf, twl);
  const double s = I.s, se2 = I.se2, inv = I.inv_ntot;
  // wave numbers of this thread's column: kx, and ky in 3D (2D: ky = line index)
  const int c = threadIdx.x % W;
  const bool live = c < cs.ncols;
  const int kx = nyq ? N / 2 : t.b + c;
  const int ky3 = nyq ? t.a + c : t.a;
  const double wgt = (kx == 0 || 2 * kx == N) ? 1.0 : 2.0;
  const double wgt_inv = wgt * inv;
  const double Kc = Sl[live ? kx : 0] + (dim == 3 ? Sl[live ? ky3 : 0] : 0.0);
  // a thread's elements lie in its column c, rows threadIdx.x / W + i * (PSD_NT / W)
  constexpr int RPT = (W * N + PSD_NT - 1) / PSD_NT;
#pragma unroll 4
  for (int i = 0; i < (live ? RPT : 0); ++i) {
    const int tt = threadIdx.x / W + i * (PSD_NT / W);
    if (W * N % PSD_NT != 0 && tt >= N) break;
    const double K = Kc + Sl[tt];
    if constexpr (OP != OP_PRECOND6) {
      buf[c * LS + pidx(tt)] = spec_one<T, OP>(buf[c * LS + pidx(tt)], K, s, se2, inv, wgt_inv, acc[0],
                                               s * I.lam);
    } else {
      const cx<T> X2 = buf[c * LS + pidx(tt)], X1 = buf[(W + c) * LS + pidx(tt)];
      if (K > 0.0) {
        const double iK = 1.0 / K;
        const double sig = s * I.lam + s * K + se2 * K * K + iK;
        const double isig = 1.0 / sig;
        const double px = (double)X2.x + iK * X1.x, py = (double)X2.y + iK * X1.y;
        const double dx = px * isig, dy = py * isig;
        acc[0] += wgt * (px * px + py * py) * isig * inv;
        acc[1] += wgt * (dx * dx + dy * dy) * iK * inv;
        buf[c * LS + pidx(tt)] = mk((T)(dx * inv), (T)(dy * inv));
        buf[(W + c) * LS + pidx(tt)] = mk((T)(X1.x * iK * inv), (T)(X1.y * iK * inv));
        buf[(2 * W + c) * LS + pidx(tt)] = mk((T)(dx * iK * inv), (T)(dy * iK * inv));
      } else {
        buf[c * LS + pidx(tt)] = mk(T(0), T(0));
        buf[(W + c) * LS + pidx(tt)] = mk(T(0), T(0));
        buf[(2 * W + c) * LS + pidx(tt)] = mk(T(0), T(0));
      }
    }
  }
  __syncthreads();
  lds_fft<T, N, NFO * W, LS, 1>(buf, twl);
  col_store<T, N, W, NFO>(base, cs, fstride, buf);
}

// Last-axis pass for one field with the values in registers (four_step):
// the operator is applied where the thread holds frequencies g + N1 k.
// LDS: transpose buffer | twiddles | symbol.
template <typename T, int N, int OP>
__device__ __forceinline__ void fused_col_fs(const Inst& I, const Task2& t, cx<T>* buf, double (&acc)[2]) {
  constexpr int W = four_step_width<N>(), N1 = N / 16;
  const cx<T>* tw = (const cx<T>*)(sizeof(T) == 8 ? I.tw64 : I.tw32);
  cx<T>* base = (cx<T>*)I.spec;
  const ColSet cs = fused_cols<T, N, W>(I, t);
  const int c = threadIdx.x % W, g = threadIdx.x / W;
  const bool live = c < cs.ncols;
  cx<T> x[16];
  col_fs_load<N>(base, cs, c, g, live, x);
  cx<T>* twl = buf + 16 * FS_RS;
  double* Sl = (double*)(twl + N);
  TableStage<cx<T>, N> tws;
  TableStage<double, N> sst;
  tws.load(tw);
  sst.load(I.S);
  tws.store(twl);
  sst.store(Sl);
  __syncthreads();
  four_step<N, -1>(x, g, c, buf, twl);   // x[k] = frequency g + N1 k
  {
    const double s = I.s, se2 = I.se2, inv = I.inv_ntot;
    const bool nyq = t.c != 0;
    const int kx = nyq ? N / 2 : t.b + c;
    const int ky3 = nyq ? t.a + c : t.a;
    const double wgt = (kx == 0 || 2 * kx == N) ? 1.0 : 2.0;
    const double wgt_inv = wgt * inv;
    const double Kc = Sl[live ? kx : 0] + (I.dim == 3 ? Sl[live ? ky3 : 0] : 0.0);
    double a0 = 0.0;
#pragma unroll
    for (int k = 0; k < 16; ++k)
      x[k] = spec_one<T, OP>(x[k], Kc + Sl[g + N1 * k], s, se2, inv, wgt_inv, a0, s * I.lam);
    if (live) acc[0] += a0;
  }
  __syncthreads();   // every thread has read the forward transpose
  four_step<N, 1>(x, g, c, buf, twl);    // x[r] = point g + N1 r
  if (live) col_fs_store<N>(base, cs, c, g, x);
}

template <typename T, int OP, int N>
__device__ __forceinline__ void fused_body(const Inst& I, const Task2& t, double* smem) {
  cx<T>* buf = (cx<T>*)smem;
  double acc[2] = {0.0, 0.0};
  constexpr int NFM = (OP == OP_PRECOND6) ? 3 : 1;
  if constexpr (NFM == 1 && col_four_step<T, N>() && col_width<T, N, NFM>() == four_step_width<N>())
    fused_col_fs<T, N, OP>(I, t, buf, acc);
  else
    fused_col<T, N, col_width<T, N, NFM>(), OP>(I, t, buf, acc);
  // the FFT buffers are dead after this barrier: reuse them for the reduction
  __syncthreads();
  block_reduce<2, 0>(acc, smem);
  if (threadIdx.x == 0) {
    I.part_sp[2 * t.slot] = acc[0];
    I.part_sp[2 * t.slot + 1] = acc[1];
  }
}

template <typename T, int OP, int N>
__global__ __launch_bounds__(PSD_NT) void k_cols_fused(const Inst* __restrict__ insts,
                                                       const Task2* __restrict__ tasks, int solver) {
  extern __shared__ double smem[];
  const Task2 t = tasks[blockIdx.x];
  const Inst& I = insts[t.inst];
  if (solver && I.st->done) return;
  fused_body<T, OP, N>(I, t, smem);
}

template <typename T, int OP>
__global__ __launch_bounds__(PSD_NT) void k_cols_fused_any(const Inst* __restrict__ insts,
                                                           const Task2* __restrict__ tasks, int solver) {
  extern __shared__ double smem[];
  const Task2 t = tasks[blockIdx.x];
  const Inst& I = insts[t.inst];
  if (solver && I.st->done) return;
  switch (I.n) {
#define PSD_C(NN) case NN: fused_body<T, OP, NN>(I, t, smem); break;
    PSD_FOR_EACH_N(PSD_C)
#undef PSD_C
    default: break;
  }
}

// ===========================================================================
// auxiliary kernels (not on the hot loop)
// ===========================================================================
// Energy partials per block (one thread per cell, direct global reads):
// [0] sum (u-f)^2  [1] sum_V |G|^p  [2] sum (Delta_h u)^2  [3] sum u^2  [4] sum u f
__global__ __launch_bounds__(PSD_NT) void k_energy_parts(const Inst* __restrict__ insts, int inst,
                                                         const double* __restrict__ u,
                                                         const double* __restrict__ f,
                                                         double* __restrict__ part) {
  __shared__ double scratch[5 * PSD_NT / PSD_WAVE];
  const Inst& I = insts[inst];
  const long long N = I.ncell;
  const int n = I.n;
  double acc[5] = {0, 0, 0, 0, 0};
  const double ih = I.inv_h, ih2 = ih * ih;
  for (long long c = blockIdx.x * (long long)PSD_NT + threadIdx.x; c < N; c += (long long)gridDim.x * PSD_NT) {
    const int i = (int)(c % n);
    const int j = (int)((c / n) % n);
    const int k = (I.dim == 3) ? (int)(c / ((long long)n * n)) : 0;
    auto at = [&](int di, int dj, int dk) -> double {
      const int ii = wrapi(i + di, n), jj = wrapi(j + dj, n), kk = (I.dim == 3) ? wrapi(k + dk, n) : 0;
      return u[ii + (long long)n * (jj + (long long)n * kk)];
    };
    const double uc = u[c];
    const double fc = f[c];
    acc[0] += (uc - fc) * (uc - fc);
    acc[3] += uc * uc;
    acc[4] += uc * fc;
    double lap = at(1, 0, 0) + at(-1, 0, 0) + at(0, 1, 0) + at(0, -1, 0) - 4.0 * uc;
    if (I.dim == 3) lap += at(0, 0, 1) + at(0, 0, -1) - 2.0 * uc;
    lap *= ih2;
    acc[2] += lap * lap;
    double g2;
    if (I.dim == 2) {
      const double c10 = at(1, 0, 0), c01 = at(0, 1, 0), c11 = at(1, 1, 0);
      const double gx = 0.5 * ih * ((c10 - uc) + (c11 - c01)), gy = 0.5 * ih * ((c01 - uc) + (c11 - c10));
      g2 = gx * gx + gy * gy;
    } else {
      const double c100 = at(1, 0, 0), c010 = at(0, 1, 0), c110 = at(1, 1, 0);
      const double c001 = at(0, 0, 1), c101 = at(1, 0, 1), c011 = at(0, 1, 1), c111 = at(1, 1, 1);
      const double q = 0.25 * ih;
      const double gx = q * ((c100 - uc) + (c110 - c010) + (c101 - c001) + (c111 - c011));
      const double gy = q * ((c010 - uc) + (c110 - c100) + (c011 - c001) + (c111 - c101));
      const double gz = q * ((c001 - uc) + (c101 - c100) + (c011 - c010) + (c111 - c110));
      g2 = gx * gx + gy * gy + gz * gz;
    }
    acc[1] += I.p_is_4 ? g2 * g2 : (I.p_is_6 ? g2 * g2 * g2 : pow(g2, 0.5 * I.p));
  }
  block_reduce<5, 0>(acc, scratch);
  if (threadIdx.x == 0)
    for (int q = 0; q < 5; ++q) part[5 * blockIdx.x + q] = acc[q];
}

// per-block sums of up to 3 fields: [0] sum a, [1] sum b, [2] sum a*b
__global__ __launch_bounds__(PSD_NT) void k_sums(const double* __restrict__ a, const double* __restrict__ b,
                                                 long long N, double* __restrict__ part) {
  __shared__ double scratch[3 * PSD_NT / PSD_WAVE];
  double acc[3] = {0, 0, 0};
  for (long long c = blockIdx.x * (long long)PSD_NT + threadIdx.x; c < N; c += (long long)gridDim.x * PSD_NT) {
    const double av = a[c];
    const double bv = b ? b[c] : 0.0;
    acc[0] += av; acc[1] += bv; acc[2] += av * bv;
  }
  block_reduce<3, 0>(acc, scratch);
  if (threadIdx.x == 0)
    for (int q = 0; q < 3; ++q) part[3 * blockIdx.x + q] = acc[q];
}

// out = alpha * a + beta * b + gamma  (b may be null)
__global__ __launch_bounds__(PSD_NT) void k_axpby(double* __restrict__ out, const double* __restrict__ a,
                                                  const double* __restrict__ b, double alpha, double beta,
                                                  double gamma, long long N) {
  for (long long c = blockIdx.x * (long long)PSD_NT + threadIdx.x; c < N; c += (long long)gridDim.x * PSD_NT)
    out[c] = alpha * a[c] + (b ? beta * b[c] : 0.0) + gamma;
}

// ===========================================================================
// adjoint: conjugate gradients on H lam = dJ/du (H = Hessian of E_h at u*,
// second variation of Sec. 5.3), preconditioned by L_h^{-1} (FFT passes).
// Flexible (Polak-Ribiere) beta, so an FP32 preconditioner is allowed:
//   beta = z+.(r+ - r)/(r.z) = -alpha (z+.Hp)/(r.z).
// SolveState reuse: c[0] = r.z, c[1] = p.Hp, c[2] = r.r, alpha, x = beta,
// hi = stop threshold on r.r, iter = CG iterations.
// ===========================================================================
template <typename TD, typename TR, int ORDER = 4>
__global__ __launch_bounds__(PSD_NT) void k_hess2d(const Inst* __restrict__ insts,
                                                   const Task2* __restrict__ tasks) {
  extern __shared__ double smem[];
  const Task2 t = tasks[blockIdx.x];
  const Inst& I = insts[t.inst];
  if (I.st->done) return;
  double acc[2] = {0.0, 0.0};
  res2d_tile<TD, TR, ORDER, false, true>(I, t.a, t.b, smem, acc);
  block_reduce<2, 1>(acc, smem + R2_LDS);
  if (threadIdx.x == 0) {
    I.part_res[2 * t.slot] = 0.0;
    I.part_res[2 * t.slot + 1] = acc[1];
  }
}

template <typename TR, int TX>
__global__ __launch_bounds__(PSD_NT) void k_hess3d(const Inst* __restrict__ insts,
                                                   const Task2* __restrict__ tasks) {
  extern __shared__ double smem[];
  const Task2 t = tasks[blockIdx.x];
  const Inst& I = insts[t.inst];
  if (I.st->done) return;
  double acc[2] = {0.0, 0.0};
  res3d_tile<double, TR, false, true, 0, TX>(I, t.a, t.b, t.c, smem, acc);
  block_reduce<2, 1>(acc, smem + R3Shape<TX>::HLDS);
  if (threadIdx.x == 0) {
    I.part_res[2 * t.slot] = 0.0;
    I.part_res[2 * t.slot + 1] = acc[1];
  }
}

// sixth-order Hessian stencil part in 3D (brick tiles): s lam xi - s div(F_lin) + s eps^2 Delta^2 xi
__global__ __launch_bounds__(PSD_NT) void k_hess3d6(const Inst* __restrict__ insts,
                                                    const Task2* __restrict__ tasks) {
  extern __shared__ double smem[];
  const Task2 t = tasks[blockIdx.x];
  const Inst& I = insts[t.inst];
  if (I.st->done) return;
  double acc[2] = {0.0, 0.0};
  res3d6_tile<double, double, false, true>(I, t.a, t.b, t.c, smem, acc);
  block_reduce<2, 1>(acc, smem + B6_LDS);
  if (threadIdx.x == 0) {
    I.part_res[2 * t.slot] = 0.0;
    I.part_res[2 * t.slot + 1] = acc[1];
  }
}

// Conjugate gradients of the sixth-order adjoint (mean-zero space, FP64):
// H Lam = P0 G with H xi = [stencil part] + T_h xi, preconditioned by the
// one-field sixth-order L_h^{-1}; tmp carries the FFT input/output (z, T_h p).
// Vector steps (block b: partials part_res[2b], part_res[2b+1]):
//   op 0: sum G                          op 1: r = G - mean, lam = 0, tmp = r; sum r.r
//   op 2: sum r.z (z = tmp)              op 3: p = z
//   op 4: tmp = p                        op 5: Hp += tmp (T_h p); sum p.Hp
//   op 6: lam += alpha p, r -= alpha Hp, tmp = r; sum r.r
//   op 7: sum r.z, sum z.Hp              op 8: p = z + beta p
// State (auxiliary): lo = mean of G, c[0] = r.z, c[1] = p.Hp, c[2] = r.r,
// hi = stop threshold, alpha, x = beta, iter = CG iterations.
__global__ __launch_bounds__(PSD_NT) void k_cg6_vec(const Inst* __restrict__ insts, int nmax, int op) {
  __shared__ double scratch[2 * PSD_NT / PSD_WAVE];
  // one launch for every instance: block (inst, j), j < nblk_vec of the instance
  const int inst = blockIdx.x / nmax, j = blockIdx.x - inst * nmax;
  const Inst& I = insts[inst];
  const SolveState* st = I.st;
  if (st->done || j >= I.nblk_vec) return;
  const long long N = I.ncell;
  const long long chunk = (N + I.nblk_vec - 1) / I.nblk_vec;
  const long long c0 = j * chunk;
  const long long c1 = c0 + chunk < N ? c0 + chunk : N;
  const double alpha = st->alpha, beta = st->x, mean = st->lo;
  double acc[2] = {0.0, 0.0};
  double* z = I.tmp;
  for (long long c = c0 + threadIdx.x; c < c1; c += PSD_NT) {
    switch (op) {
      case 0: acc[1] += I.adj_g[c]; break;
      case 1: {
        const double r = I.adj_g[c] - mean;
        I.adj_r[c] = r; I.adj_lam[c] = 0.0; z[c] = r; acc[1] += r * r;
      } break;
      case 2: acc[1] += I.adj_r[c] * z[c]; break;
      case 3: I.adj_p[c] = z[c]; break;
      case 4: z[c] = I.adj_p[c]; break;
      case 5: {
        const double hp = I.adj_Hp[c] + z[c];
        I.adj_Hp[c] = hp; acc[1] += I.adj_p[c] * hp;
      } break;
      case 6: {
        I.adj_lam[c] += alpha * I.adj_p[c];
        const double r = I.adj_r[c] - alpha * I.adj_Hp[c];
        I.adj_r[c] = r; z[c] = r; acc[1] += r * r;
      } break;
      case 7: acc[0] += I.adj_r[c] * z[c]; acc[1] += z[c] * I.adj_Hp[c]; break;
      default: I.adj_p[c] = z[c] + beta * I.adj_p[c]; break;
    }
  }
  if (op == 0 || op == 1 || op == 2 || op == 5 || op == 6 || op == 7) {
    block_reduce<2, 0>(acc, scratch);
    if (threadIdx.x == 0) { I.part_res[2 * j] = acc[0]; I.part_res[2 * j + 1] = acc[1]; }
  }
}

// One block per instance: reduce the nblk_vec vector partials and update the
// scalars of k_cg6_vec.  mode 0: mean of G; 1: threshold; 2: r.z; 3: alpha;
// 4: r.r and stop test; 5: beta and the new r.z.
__global__ __launch_bounds__(PSD_NT) void k_cg6_fin(const Inst* __restrict__ insts, int mode, double rtol2) {
  __shared__ double scratch[2 * PSD_NT / PSD_WAVE];
  const Inst& I = insts[blockIdx.x];
  SolveState* st = I.st;
  if (st->done) return;
  double acc[2] = {0.0, 0.0};
  for (int b = threadIdx.x; b < I.nblk_vec; b += PSD_NT) {
    acc[0] += I.part_res[2 * b];
    acc[1] += I.part_res[2 * b + 1];
  }
  block_reduce<2, 0>(acc, scratch);
  if (threadIdx.x != 0) return;
  if (mode == 0) {
    st->lo = acc[1] * I.inv_ntot;
  } else if (mode == 1) {
    st->hi = rtol2 * acc[1];
    st->c[2] = acc[1];
    if (!(acc[1] > 0.0)) st->done = 1;   // G constant: Lam = 0
  } else if (mode == 2) {
    st->c[0] = acc[1];
  } else if (mode == 3) {
    st->c[1] = acc[1];
    if (!(acc[1] > 0.0)) { st->status = -5; st->done = 1; return; }
    st->alpha = st->c[0] / acc[1];
  } else if (mode == 4) {
    st->c[2] = acc[1];
    st->iter += 1;
    if (!isfinite(acc[1])) { st->status = -4; st->done = 1; }
    else if (acc[1] <= st->hi) st->done = 1;
    else if (st->iter >= I.max_iter) { st->status = 1; st->done = 1; }
  } else {
    st->x = -st->alpha * acc[1] / st->c[0];
    st->c[0] = acc[0];
  }
}

// Vector steps over the cells of one instance; block b handles a contiguous
// chunk and writes one partial sum to part_res[2b+1].
//   op 0: lam = 0, r = g, rTR = g;            partial g.g
//   op 1: lam += alpha p, r -= alpha Hp, rTR = r;  partial r.r
//   op 2: partial z.Hp
//   op 3: p = z (first) ; op 4: p = z + beta p
template <typename TD, typename TR>
__global__ __launch_bounds__(PSD_NT) void k_cg_vec(const Inst* __restrict__ insts, int nmax, int op) {
  __shared__ double scratch[2 * PSD_NT / PSD_WAVE];
  // one launch for every instance: block (inst, j), j < nblk_vec of the instance
  const int inst = blockIdx.x / nmax, j = blockIdx.x - inst * nmax;
  const Inst& I = insts[inst];
  const SolveState* st = I.st;
  if (st->done || j >= I.nblk_vec) return;
  const long long N = I.ncell;
  const long long chunk = (N + I.nblk_vec - 1) / I.nblk_vec;
  const long long c0 = j * chunk;
  const long long c1 = c0 + chunk < N ? c0 + chunk : N;
  const double alpha = st->alpha, beta = st->x;
  double acc[2] = {0.0, 0.0};
  const TD* z = (const TD*)I.d;
  TR* rtr = (TR*)I.r;
  for (long long c = c0 + threadIdx.x; c < c1; c += PSD_NT) {
    if (op == 0) {
      const double g = I.adj_g[c];
      I.adj_lam[c] = 0.0;
      I.adj_r[c] = g;
      rtr[c] = (TR)g;
      acc[1] += g * g;
    } else if (op == 1) {
      I.adj_lam[c] += alpha * I.adj_p[c];
      const double r = I.adj_r[c] - alpha * I.adj_Hp[c];
      I.adj_r[c] = r;
      rtr[c] = (TR)r;
      acc[1] += r * r;
    } else if (op == 2) {
      acc[1] += (double)z[c] * I.adj_Hp[c];
    } else if (op == 3) {
      I.adj_p[c] = (double)z[c];
    } else {
      I.adj_p[c] = (double)z[c] + beta * I.adj_p[c];
    }
  }
  if (op <= 2) {
    block_reduce<2, 1>(acc, scratch);
    if (threadIdx.x == 0) I.part_res[2 * j + 1] = acc[1];
  }
}

// One block per instance.  mode 0: threshold from g.g; 1: r.z from the
// spectral partials; 2: alpha = r.z / p.Hp; 3: r.r and stop test; 4: beta.
__global__ __launch_bounds__(PSD_NT) void k_cg_fin(const Inst* __restrict__ insts, int mode, int nblk_vec,
                                                   double rtol2) {
  __shared__ double scratch[2 * PSD_NT / PSD_WAVE];
  const Inst& I = insts[blockIdx.x];
  SolveState* st = I.st;
  if (st->done) return;
  double acc[2] = {0.0, 0.0};
  if (mode == 1 || mode == 4)
    for (int b = threadIdx.x; b < I.nblk_sp; b += PSD_NT) acc[0] += I.part_sp[2 * b];
  // mode 2 reduces the Hessian pass (one partial per residual tile), the
  // others the vector kernels (nblk_vec partials, or the count given)
  const int nb = mode == 2 ? I.nblk_res : (nblk_vec < 0 ? I.nblk_vec : nblk_vec);
  if (mode != 1)
    for (int b = threadIdx.x; b < nb; b += PSD_NT) acc[1] += I.part_res[2 * b + 1];
  block_reduce<2, 0>(acc, scratch);
  if (threadIdx.x != 0) return;
  if (mode == 0) {
    st->hi = rtol2 * acc[1];
    st->c[2] = acc[1];
    if (!(acc[1] > 0.0)) st->done = 1;   // zero right-hand side: lam = 0
  } else if (mode == 1) {
    st->c[0] = acc[0];
  } else if (mode == 2) {
    st->c[1] = acc[1];
    if (!(acc[1] > 0.0)) { st->status = -5; st->done = 1; return; }
    st->alpha = st->c[0] / acc[1];
  } else if (mode == 3) {
    st->c[2] = acc[1];
    st->iter += 1;
    if (!isfinite(acc[1])) { st->status = -4; st->done = 1; }
    else if (acc[1] <= st->hi) st->done = 1;
    else if (st->iter >= I.max_iter) { st->status = 1; st->done = 1; }
  } else {
    const double rz_new = acc[0];
    st->x = -st->alpha * acc[1] / st->c[0];
    st->c[0] = rz_new;
  }
}

// Parameter sensitivities of N_h at u* weighted by lam (one thread per cell,
// direct reads):  part[3b] = sum lam (-plap u* + eps^2 Delta_h^2 u*),
// part[3b+1] = sum lam Delta_h^2 u*, part[3b+2] = sum lam u*.
__device__ __forceinline__ double at3(const double* u, int n, int dim, int i, int j, int k) {
  i = wrapi(i, n); j = wrapi(j, n);
  k = dim == 3 ? wrapi(k, n) : 0;
  return u[i + (long long)n * (j + (long long)n * k)];
}

// div_h(R grad_h u) at cell (i, j, k) from the 4 (2D) or 8 (3D) vertices
// around it, with R = |grad_h u|^{p-2} (linear = false) or R = 1 (linear =
// true: the skew Laplacian Delta_h^v of Sec. 5.1); direct global reads.
__device__ __forceinline__ double div_flux_at(const Inst& I, const double* u, int i, int j, int k,
                                              bool linear) {
  const int n = I.n, dim = I.dim;
  const double ih = I.inv_h;
  double div = 0.0;
  const int nz = dim == 3 ? 2 : 1;
  for (int cz = 0; cz < nz; ++cz)
    for (int cy = 0; cy < 2; ++cy)
      for (int cx = 0; cx < 2; ++cx) {
        // vertex (i - 1 + cx + 1/2, j - 1 + cy + 1/2, k - 1 + cz + 1/2): lower cell corner
        const int vi = i - 1 + cx, vj = j - 1 + cy, vk = dim == 3 ? k - 1 + cz : 0;
        double gx, gy, gz = 0.0;
        if (dim == 2) {
          const double c00 = at3(u, n, 2, vi, vj, 0), c10 = at3(u, n, 2, vi + 1, vj, 0);
          const double c01 = at3(u, n, 2, vi, vj + 1, 0), c11 = at3(u, n, 2, vi + 1, vj + 1, 0);
          gx = 0.5 * ih * ((c10 - c00) + (c11 - c01));
          gy = 0.5 * ih * ((c01 - c00) + (c11 - c10));
        } else {
          const double c000 = at3(u, n, 3, vi, vj, vk), c100 = at3(u, n, 3, vi + 1, vj, vk);
          const double c010 = at3(u, n, 3, vi, vj + 1, vk), c110 = at3(u, n, 3, vi + 1, vj + 1, vk);
          const double c001 = at3(u, n, 3, vi, vj, vk + 1), c101 = at3(u, n, 3, vi + 1, vj, vk + 1);
          const double c011 = at3(u, n, 3, vi, vj + 1, vk + 1), c111 = at3(u, n, 3, vi + 1, vj + 1, vk + 1);
          const double q = 0.25 * ih;
          gx = q * ((c100 - c000) + (c110 - c010) + (c101 - c001) + (c111 - c011));
          gy = q * ((c010 - c000) + (c110 - c100) + (c011 - c001) + (c111 - c101));
          gz = q * ((c001 - c000) + (c101 - c100) + (c011 - c010) + (c111 - c110));
        }
        const double rr = linear ? 1.0 : flux_r(gx * gx + gy * gy + gz * gz, I.p, I.p_is_4, I.p_is_2);
        // divergence weights: +-1/(2h) (2D) or +-1/(4h) (3D) per component
        const double w = dim == 2 ? 0.5 * ih : 0.25 * ih;
        div += w * ((cx ? 1.0 : -1.0) * rr * gx + (cy ? 1.0 : -1.0) * rr * gy +
                    (dim == 3 ? (cz ? 1.0 : -1.0) * rr * gz : 0.0));
      }
  return div;
}

// Parameter sensitivities of the adjoint: with lam = H^{-1} dJ/du,
//   part[0] = sum_c lam (-div_h F(u*) + eps^2 Delta_h^2 u*),  F = |grad u|^{p-2} grad u,
//   part[1] = sum_c lam Delta_h^2 u*,  part[2] = sum_c lam u*,
// evaluated by summation by parts (the vertex gradient is minus the adjoint
// of the divergence, Delta_h is self-adjoint): sum_c lam (-div F) =
// sum_v grad lam . F and sum_c lam Delta_h^2 u = sum_c Delta_h lam Delta_h u.
// Each cell contributes its upper vertex (i+1/2, j+1/2[, k+1/2]) and its own
// Laplacians: 16 (3D) loads of u and lam for the vertex, 12 for the
// Laplacians.
__global__ __launch_bounds__(PSD_NT) void k_param_sens(const Inst* __restrict__ insts, int inst,
                                                       double* __restrict__ part) {
  __shared__ double scratch[3 * PSD_NT / PSD_WAVE];
  const Inst& I = insts[inst];
  const double* u = I.adj_us;
  const double* lm = I.adj_lam;
  const int n = I.n, dim = I.dim;
  const double ih = I.inv_h, ih2 = ih * ih;
  const double e2 = I.se2 / I.s;
  double acc[3] = {0.0, 0.0, 0.0};
  for (long long c = blockIdx.x * (long long)PSD_NT + threadIdx.x; c < I.ncell; c += (long long)gridDim.x * PSD_NT) {
    const int i = (int)(c % n), j = (int)((c / n) % n), k = dim == 3 ? (int)(c / ((long long)n * n)) : 0;
    double gx, gy, gz = 0.0, hx, hy, hz = 0.0;   // grad u*, grad lam at the vertex
    if (dim == 2) {
      const double c00 = at3(u, n, 2, i, j, 0), c10 = at3(u, n, 2, i + 1, j, 0);
      const double c01 = at3(u, n, 2, i, j + 1, 0), c11 = at3(u, n, 2, i + 1, j + 1, 0);
      gx = 0.5 * ih * ((c10 - c00) + (c11 - c01));
      gy = 0.5 * ih * ((c01 - c00) + (c11 - c10));
      const double l00 = at3(lm, n, 2, i, j, 0), l10 = at3(lm, n, 2, i + 1, j, 0);
      const double l01 = at3(lm, n, 2, i, j + 1, 0), l11 = at3(lm, n, 2, i + 1, j + 1, 0);
      hx = 0.5 * ih * ((l10 - l00) + (l11 - l01));
      hy = 0.5 * ih * ((l01 - l00) + (l11 - l10));
    } else {
      const double q = 0.25 * ih;
      const double c000 = at3(u, n, 3, i, j, k), c100 = at3(u, n, 3, i + 1, j, k);
      const double c010 = at3(u, n, 3, i, j + 1, k), c110 = at3(u, n, 3, i + 1, j + 1, k);
      const double c001 = at3(u, n, 3, i, j, k + 1), c101 = at3(u, n, 3, i + 1, j, k + 1);
      const double c011 = at3(u, n, 3, i, j + 1, k + 1), c111 = at3(u, n, 3, i + 1, j + 1, k + 1);
      gx = q * ((c100 - c000) + (c110 - c010) + (c101 - c001) + (c111 - c011));
      gy = q * ((c010 - c000) + (c110 - c100) + (c011 - c001) + (c111 - c101));
      gz = q * ((c001 - c000) + (c101 - c100) + (c011 - c010) + (c111 - c110));
      const double l000 = at3(lm, n, 3, i, j, k), l100 = at3(lm, n, 3, i + 1, j, k);
      const double l010 = at3(lm, n, 3, i, j + 1, k), l110 = at3(lm, n, 3, i + 1, j + 1, k);
      const double l001 = at3(lm, n, 3, i, j, k + 1), l101 = at3(lm, n, 3, i + 1, j, k + 1);
      const double l011 = at3(lm, n, 3, i, j + 1, k + 1), l111 = at3(lm, n, 3, i + 1, j + 1, k + 1);
      hx = q * ((l100 - l000) + (l110 - l010) + (l101 - l001) + (l111 - l011));
      hy = q * ((l010 - l000) + (l110 - l100) + (l011 - l001) + (l111 - l101));
      hz = q * ((l001 - l000) + (l101 - l100) + (l011 - l010) + (l111 - l110));
    }
    const double rr = flux_r(gx * gx + gy * gy + gz * gz, I.p, I.p_is_4, I.p_is_2);
    auto lap = [&](const double* v) {
      double t = at3(v, n, dim, i + 1, j, k) + at3(v, n, dim, i - 1, j, k) + at3(v, n, dim, i, j + 1, k) +
                 at3(v, n, dim, i, j - 1, k) - 4.0 * at3(v, n, dim, i, j, k);
      if (dim == 3) t += at3(v, n, dim, i, j, k + 1) + at3(v, n, dim, i, j, k - 1) - 2.0 * at3(v, n, dim, i, j, k);
      return t * ih2;
    };
    const double ll = lap(lm) * lap(u);
    acc[0] += rr * (hx * gx + hy * gy + hz * gz) + e2 * ll;
    acc[1] += ll;
    acc[2] += lm[c] * u[c];
  }
  block_reduce<3, 0>(acc, scratch);
  if (threadIdx.x == 0)
    for (int q = 0; q < 3; ++q) part[3 * blockIdx.x + q] = acc[q];
}

// Right-hand sides of the convex-splitting time steps from the current time
// level u (one thread per cell):
//   scheme 0, thin film (Sec. 6.1):  f = u - s Delta_h^v u   (skew Laplacian)
//   scheme 1, SPFC (Sec. 6.2):       g = u,  f = -s gamma1 Delta_h u   (5-point;
//                                    s makes the step consistent with the H^-1 flow)
__global__ __launch_bounds__(PSD_NT) void k_ts_rhs(const Inst* __restrict__ insts, int inst, int scheme,
                                                   double gamma1, const double* __restrict__ u,
                                                   double* __restrict__ f, double* __restrict__ g) {
  const Inst& I = insts[inst];
  const int n = I.n, dim = I.dim;
  const double ih2 = I.inv_h * I.inv_h;
  for (long long c = blockIdx.x * (long long)PSD_NT + threadIdx.x; c < I.ncell; c += (long long)gridDim.x * PSD_NT) {
    const int i = (int)(c % n), j = (int)((c / n) % n), k = dim == 3 ? (int)(c / ((long long)n * n)) : 0;
    const double uc = u[c];
    if (scheme == 0) {
      f[c] = uc - I.s * div_flux_at(I, u, i, j, k, true);
    } else {
      double lap = at3(u, n, dim, i + 1, j, k) + at3(u, n, dim, i - 1, j, k) + at3(u, n, dim, i, j + 1, k) +
                   at3(u, n, dim, i, j - 1, k) - 4.0 * uc;
      if (dim == 3) lap += at3(u, n, dim, i, j, k + 1) + at3(u, n, dim, i, j, k - 1) - 2.0 * uc;
      f[c] = -I.s * gamma1 * lap * ih2;
      g[c] = uc;
    }
  }
}

// Variable metric: the conjugate-gradient solution x = L_k^{-1} r (FP64, in
// I.adj_lam) becomes the search direction d (TD), and each block writes the
// partial sum of r.d (r = I.adj_g, the FP64 residual) into the spectral
// partial slot the line-search finalize reads for -q(0) (block b of nblk_sp,
// grid-stride over the cells).
template <typename TD>
__global__ __launch_bounds__(PSD_NT) void k_vm_finish(const Inst* __restrict__ insts, int inst) {
  __shared__ double scratch[2 * PSD_NT / PSD_WAVE];
  const Inst& I = insts[inst];
  if (I.st->done) return;
  TD* d = (TD*)I.d;
  double acc[2] = {0.0, 0.0};
  for (long long c = blockIdx.x * (long long)PSD_NT + threadIdx.x; c < I.ncell; c += (long long)gridDim.x * PSD_NT) {
    const TD dv = (TD)I.adj_lam[c];
    d[c] = dv;
    acc[0] += I.adj_g[c] * (double)dv;
  }
  block_reduce<2, 0>(acc, scratch);
  if (threadIdx.x == 0) {
    I.part_sp[2 * blockIdx.x] = acc[0];
    I.part_sp[2 * blockIdx.x + 1] = 0.0;
  }
}

// Variable metric: FP64 copy of the residual (the right-hand side of the
// direction solve) and done flags of the finished solves copied to the
// conjugate-gradient states.
template <typename TR>
__global__ __launch_bounds__(PSD_NT) void k_vm_start(const Inst* __restrict__ insts, int inst,
                                                     const SolveState* __restrict__ psd_st) {
  const Inst& I = insts[inst];
  if (blockIdx.x == 0 && threadIdx.x == 0 && psd_st[inst].done) I.st->done = 1;
  if (psd_st[inst].done) return;
  const TR* r = (const TR*)I.r;
  double* g = const_cast<double*>(I.adj_g);
  for (long long c = blockIdx.x * (long long)PSD_NT + threadIdx.x; c < I.ncell; c += (long long)gridDim.x * PSD_NT)
    g[c] = (double)r[c];
}

// mark every instance except `keep` as finished (auxiliary single-instance calls)
__global__ void k_mark_done(const Inst* __restrict__ insts, int ninst, int keep) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < ninst && i != keep) insts[i].st->done = 1;
}

__global__ void k_set_status(const Inst* __restrict__ insts, int inst, int status) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    insts[inst].st->status = status;
    insts[inst].st->done = 1;
  }
}

__global__ void k_reset_state(const Inst* __restrict__ insts, int ninst) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= ninst) return;
  SolveState* st = insts[i].st;
  st->alpha = 0.0; st->rinf = 0.0; st->rl2 = 0.0;
  for (int k = 0; k < 4; ++k) st->c[k] = 0.0;
  st->iter = 0; st->done = 0; st->status = 0; st->ls_phase = 0; st->dE = 0.0; st->ls_trunc = 0;
  st->mean[0] = st->mean[1] = st->mean[2] = 0.0;
}

}  // namespace psd
