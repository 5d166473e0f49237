// psd_common.hpp -- shared device types for the gfx950 PSD solver.
//
// Layout conventions (Sec. 5.1 of the paper): periodic n^dim cell-centred
// grid, x fastest, idx = i + n*(j + n*k).  A vertex (i+1/2, j+1/2[, k+1/2])
// is addressed by the index of cell (i, j[, k]).  Spectra are half spectra
// (kx = 0 .. n/2).  A field holds the columns kx < n/2 as rows [kz][ky][kx],
// kx fastest, row stride ncp (n/2 rounded up to 128 bytes), followed by the
// Nyquist plane kx = n/2 stored [kz][ky] (offset nyq): every row is a whole
// number of 128-byte lines and no padding column is ever read or written.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#define PSD_NT 256          // threads per block for every kernel
#define PSD_WAVE 64         // gfx950 wavefront

namespace psd {

template <typename T>
struct alignas(2 * sizeof(T)) cx {
  T x, y;
};

template <typename T>
__device__ __forceinline__ cx<T> mk(T a, T b) { cx<T> r; r.x = a; r.y = b; return r; }
template <typename T>
__device__ __forceinline__ cx<T> operator+(cx<T> a, cx<T> b) { return mk(a.x + b.x, a.y + b.y); }
template <typename T>
__device__ __forceinline__ cx<T> operator-(cx<T> a, cx<T> b) { return mk(a.x - b.x, a.y - b.y); }
template <typename T>
__device__ __forceinline__ cx<T> operator*(cx<T> a, cx<T> b) {
  return mk(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
template <typename T>
__device__ __forceinline__ cx<T> scale(cx<T> a, T s) { return mk(a.x * s, a.y * s); }
template <typename T>
__device__ __forceinline__ cx<T> conj(cx<T> a) { return mk(a.x, -a.y); }
// multiply by +i (DIR = +1) or -i (DIR = -1)
template <int DIR, typename T>
__device__ __forceinline__ cx<T> mul_i(cx<T> a) {
  return DIR > 0 ? mk(-a.y, a.x) : mk(a.y, -a.x);
}

// ---------------------------------------------------------------------------
// Per-instance descriptor (device resident).  Field pointers are typed by
// the precision form: TD = type of d/e1/e2, TR = type of the residual copy
// given to the FFT (FP64 form: double, mixed form: float).
// ---------------------------------------------------------------------------
struct SolveState {
  double alpha;        // current line-search step
  double rinf, rl2;    // max-norm and l2 (h^dim weighted) of the last residual
  double c[6];         // polynomial coefficients of q (p = 4: cubic, p = 6: quintic)
                       // or q(0), q'(0) (general p)
  double lin;          // general p: linear part of q'
  double nl0;          // general p: nonlinear vertex sum at alpha = 0
  double lo, hi, x, qx, dqx;  // root-rule state (general p)
  int iter;            // updates applied so far
  int done;            // 1: converged / stopped (kernels early-exit)
  int status;          // psd_status
  int ls_phase;        // general p root rule: 1 searching, 2 finished
  int ls_evals;
  int newton_steps;
  double dE;           // energy decrease of the last step (p = 4)
  double mean[3];      // order 6: means of d, e1, e2 removed in the update
  int ls_trunc;        // general p: line searches stopped by the evaluation cap
  int pad1;
};

struct Inst {
  int dim, n, nc, order;
  long long ncell;     // n^dim
  long long nspec;     // largest field stride of the spectrum buffer (complex elements)
  int ncp32, ncp64;    // spectrum row strides (kx < n/2, 128-byte multiples) for FP32 / FP64
  long long nspec32, nspec64;  // spectrum field strides (complex elements)
  long long nyq32, nyq64;      // offset of the Nyquist plane in a field = ncp * n^(dim-1)
  double h, inv_h, p, s, se2, lam, inv_ntot, tol, hd;
  int max_iter, p_is_4, p_is_2, p_is_6;
  double* u[2];        // ping-pong iterate
  double* w[2];        // order 6 carried w (ping-pong)
  const double* f;
  const double* g;
  void* d;             // search direction (TD)
  void* e1;            // order 6: T_h r1 (TD)
  void* e2;            // order 6: T_h d (TD)
  void* r;             // residual copy for the FFT (TR); order 6: r2
  void* r1;            // order 6: r1 (TR)
  void* spec;          // half spectra, up to 3 fields of nspec complex
  const double* S;     // S[k] = (4/h^2) sin^2(pi k/n), k in [0,n)
  const void* tw32;    // twiddles exp(-2 pi i m/n), m in [0,n), FP32 complex
  const void* tw64;    // the same in FP64 complex
  double* tmp;         // FP64 scratch field (auxiliary transforms)
  SolveState* st;
  double* part_res;    // residual partials: 2 per block (max|r|, sum r^2)
  double* part_ls;     // line-search partials: 8 per block
  double* part_sp;     // spectral partials: 2 per block
  double* part_c2r;    // sums of the inverse-transform outputs: 3 per block
  double* hist;        // 4 per update (may be null)
  // adjoint (conjugate gradients on the Hessian of E_h at u*)
  const double* adj_us;   // u*
  const double* adj_g;    // right-hand side dJ/du
  double* adj_lam;        // solution (= dJ/df)
  double* adj_r;          // CG residual
  double* adj_p;          // CG direction
  double* adj_Hp;         // Hessian times direction
  int nblk_res, nblk_ls, nblk_sp, hist_cap;
  int nblk_c2r;
  int zchunk_res;      // 3D: z-planes marched per residual block (tuned)
  int zchunk_ls;       // 3D: z-planes marched per line-search block (tuned)
  int nblk_vec;        // blocks of the adjoint's vector kernels (and their partials)
  int adj_frozen;      // 1: the operator of the conjugate gradients is the variable
                       // metric L_k (frozen p-Laplacian coefficient), not the Hessian
};

// A block's unit of work: instance and up to three integer coordinates.
struct Task {
  int inst, a, b, c;
};

// ---------------------------------------------------------------------------
// Block reductions (wavefront shuffles, then LDS across the 4 waves).
// Deterministic: fixed shuffle tree and fixed order across waves.
// ---------------------------------------------------------------------------
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = PSD_WAVE / 2; o > 0; o >>= 1) v += __shfl_xor(v, o, PSD_WAVE);
  return v;
}
__device__ __forceinline__ double wave_max(double v) {
#pragma unroll
  for (int o = PSD_WAVE / 2; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, PSD_WAVE));
  return v;
}

// Reduce K sums (and optionally the first M as max instead) across the
// block; result valid in thread 0.  scratch: K * (NT/64) doubles of LDS.
template <int K, int M, int NT = PSD_NT>
__device__ __forceinline__ void block_reduce(double (&v)[K], double* scratch) {
  const int lane = threadIdx.x & (PSD_WAVE - 1);
  const int wid = threadIdx.x / PSD_WAVE;
  constexpr int NW = NT / PSD_WAVE;
#pragma unroll
  for (int k = 0; k < K; ++k) v[k] = (k < M) ? wave_max(v[k]) : wave_sum(v[k]);
  __syncthreads();
  if (lane == 0) {
#pragma unroll
    for (int k = 0; k < K; ++k) scratch[k * NW + wid] = v[k];
  }
  __syncthreads();
  if (threadIdx.x == 0) {
#pragma unroll
    for (int k = 0; k < K; ++k) {
      double a = scratch[k * NW];
      for (int w2 = 1; w2 < NW; ++w2) a = (k < M) ? fmax(a, scratch[k * NW + w2]) : a + scratch[k * NW + w2];
      v[k] = a;
    }
  }
  __syncthreads();
}

// Global-memory view of a pointer read from a table.  Pointers taken from the
// instance table are generic to the compiler, which then issues flat memory
// instructions; those also count against the LDS wait counter, so every LDS
// wait (and every barrier) would drain all loads in flight.  Casting to the
// global address space gives global loads and stores instead.
#define PSD_GLOBAL __attribute__((address_space(1)))

// 1/x for finite x >= 1: the hardware reciprocal estimate refined by two
// Newton-Raphson steps r <- r + r (1 - x r), each of which squares the
// relative error
__device__ __forceinline__ double rcp_pos(double x) {
  double r = __builtin_amdgcn_rcp(x);
  double e = fma(-x, r, 1.0);
  r = fma(r, e, r);
  e = fma(-x, r, 1.0);
  return fma(r, e, r);
}
template <typename T>
__device__ __forceinline__ PSD_GLOBAL T* gmem(T* p) { return (PSD_GLOBAL T*)p; }
template <typename T>
__device__ __forceinline__ const PSD_GLOBAL T* gmem(const T* p) { return (const PSD_GLOBAL T*)p; }

// Native vectors for global loads and stores of small aggregates (structs
// cannot be copied to or from the global address space).
template <typename T, int K>
using gvec = T __attribute__((ext_vector_type(K)));

template <typename T>
__device__ __forceinline__ cx<T> gld(const cx<T>* p) {
  const gvec<T, 2> v = *(const PSD_GLOBAL gvec<T, 2>*)gmem(p);
  return mk(v.x, v.y);
}
// global load of a table entry, complex or real
template <typename T>
__device__ __forceinline__ cx<T> gld_any(const cx<T>* p) { return gld(p); }
__device__ __forceinline__ double gld_any(const double* p) { return *gmem(p); }

template <typename T>
__device__ __forceinline__ void gst(cx<T>* p, const cx<T>& a) {
  gvec<T, 2> v;
  v.x = a.x;
  v.y = a.y;
  *(PSD_GLOBAL gvec<T, 2>*)gmem(p) = v;
}

// Threads of the per-instance finalize kernels (one block per instance).
constexpr int PSD_FIN_NT = 1024;

// Accumulate K-wide block partials part[K*b + k], b < nblk, over the threads
// of a PSD_FIN_NT block (the first M as max, the rest as sums).  Four slots
// per thread are loaded before any is added, so the loads of a round are in
// flight together.  The order of the additions is fixed.
template <int K, int M>
__device__ __forceinline__ void gather_parts(const double* __restrict__ part, int nblk,
                                             double (&acc)[K]) {
  constexpr int U = 4;
  for (int b0 = 0; b0 < nblk; b0 += U * PSD_FIN_NT) {
    double v[U][K];
#pragma unroll
    for (int j = 0; j < U; ++j) {
      const int b = b0 + j * PSD_FIN_NT + (int)threadIdx.x;
#pragma unroll
      for (int k = 0; k < K; ++k) v[j][k] = b < nblk ? gmem(part)[K * b + k] : 0.0;
    }
#pragma unroll
    for (int j = 0; j < U; ++j)
#pragma unroll
      for (int k = 0; k < K; ++k) acc[k] = (k < M) ? fmax(acc[k], v[j][k]) : acc[k] + v[j][k];
  }
}

// Reduce K-wide block partials part[K*b + k], b < nblk, read as one flat
// array: with K a power of two dividing 64, thread t only ever sees entry
// k = t mod K, so every wave load is contiguous.  The first M entries are
// maxima of non-negative values, the rest sums.  Lanes of equal k are
// combined by a fixed butterfly, then waves in order; result in thread 0.
template <int K, int M, int NT>
__device__ __forceinline__ void flat_reduce(const double* __restrict__ part, int nblk,
                                            double (&out)[K], double* scratch) {
  static_assert((K & (K - 1)) == 0 && K <= PSD_WAVE && NT % PSD_WAVE == 0, "K | 64");
  constexpr int NW = NT / PSD_WAVE;
  constexpr int U = 8;
  const int tid = threadIdx.x, lane = tid & (PSD_WAVE - 1), wid = tid / PSD_WAVE;
  const bool is_max = (tid % K) < M;
  const int total = K * nblk;
  double a = 0.0;
  for (int j0 = 0; j0 < total; j0 += U * NT) {
    double v[U];
#pragma unroll
    for (int q = 0; q < U; ++q) {
      const int j = j0 + q * NT + tid;
      v[q] = j < total ? gmem(part)[j] : 0.0;
    }
#pragma unroll
    for (int q = 0; q < U; ++q) a = is_max ? fmax(a, v[q]) : a + v[q];
  }
#pragma unroll
  for (int o = PSD_WAVE / 2; o >= K; o >>= 1) {
    const double b = __shfl_xor(a, o, PSD_WAVE);
    a = is_max ? fmax(a, b) : a + b;
  }
  if (lane < K) scratch[wid * K + lane] = a;
  __syncthreads();
  if (tid == 0) {
#pragma unroll
    for (int k = 0; k < K; ++k) {
      double r = scratch[k];
      for (int w = 1; w < NW; ++w) r = (k < M) ? fmax(r, scratch[w * K + k]) : r + scratch[w * K + k];
      out[k] = r;
    }
  }
  __syncthreads();
}

// Two flat reductions (K1- and K2-wide sums of block partials) whose loads
// are issued together, so that both cost one memory round trip.  Results in
// thread 0.  scratch: (K1 + K2) * NT / 64 doubles.
template <int K1, int K2, int NT>
__device__ __forceinline__ void flat_reduce2(const double* __restrict__ p1, int n1,
                                             const double* __restrict__ p2, int n2,
                                             double (&o1)[K1], double (&o2)[K2], double* scratch) {
  static_assert((K1 & (K1 - 1)) == 0 && (K2 & (K2 - 1)) == 0 && K1 <= PSD_WAVE && K2 <= PSD_WAVE, "K | 64");
  constexpr int NW = NT / PSD_WAVE;
  constexpr int U = 8;
  const int tid = threadIdx.x, lane = tid & (PSD_WAVE - 1), wid = tid / PSD_WAVE;
  const int t1 = K1 * n1, t2 = K2 * n2;
  const int tmax = t1 > t2 ? t1 : t2;
  double a = 0.0, b = 0.0;
  for (int j0 = 0; j0 < tmax; j0 += U * NT) {
    double v[U], w[U];
#pragma unroll
    for (int q = 0; q < U; ++q) {
      const int j = j0 + q * NT + tid;
      v[q] = j < t1 ? gmem(p1)[j] : 0.0;
      w[q] = j < t2 ? gmem(p2)[j] : 0.0;
    }
#pragma unroll
    for (int q = 0; q < U; ++q) { a += v[q]; b += w[q]; }
  }
#pragma unroll
  for (int o = PSD_WAVE / 2; o >= K1; o >>= 1) a += __shfl_xor(a, o, PSD_WAVE);
#pragma unroll
  for (int o = PSD_WAVE / 2; o >= K2; o >>= 1) b += __shfl_xor(b, o, PSD_WAVE);
  if (lane < K1) scratch[wid * K1 + lane] = a;
  if (lane < K2) scratch[NW * K1 + wid * K2 + lane] = b;
  __syncthreads();
  // thread k < K1 + K2 adds entry k over the waves in wave order (in
  // parallel rather than all in thread 0; the order of the additions is the
  // same), then thread 0 collects the results
  static_assert(K1 + K2 <= NT, "one thread per entry");
  double r = 0.0;
  if (tid < K1) {
    r = scratch[tid];
    for (int w2 = 1; w2 < NW; ++w2) r += scratch[w2 * K1 + tid];
  } else if (tid < K1 + K2) {
    const int k = tid - K1;
    r = scratch[NW * K1 + k];
    for (int w2 = 1; w2 < NW; ++w2) r += scratch[NW * K1 + w2 * K2 + k];
  }
  __syncthreads();
  if (tid < K1 + K2) scratch[tid] = r;
  __syncthreads();
  if (tid == 0) {
#pragma unroll
    for (int k = 0; k < K1; ++k) o1[k] = scratch[k];
#pragma unroll
    for (int k = 0; k < K2; ++k) o2[k] = scratch[K1 + k];
  }
  __syncthreads();
}

// periodic index for offsets within one period (3D tiles: n >= 32 is
// required so that every halo index lies in [-n, 2n))
__device__ __forceinline__ int wrapi(int i, int n) { return i < 0 ? i + n : (i >= n ? i - n : i); }
// periodic index for any i >= -n (2D tiles may be wider than small grids)
__device__ __forceinline__ int posmod(int i, int n) { return (int)((unsigned)(i + n) % (unsigned)n); }

}  // namespace psd
