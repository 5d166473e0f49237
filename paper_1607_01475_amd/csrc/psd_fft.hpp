// psd_fft.hpp -- LDS-resident batched FFT passes for gfx950.
//
// The preconditioner L_h is diagonal in the discrete Fourier basis (Sec. 6:
// the search-direction equations are solved by FFT), so one application is
// forward transform -> divide by the symbol -> inverse transform.  Lines of
// length N (N = 2^a 3^b, 16 <= N <= 1024) are transformed inside LDS with a
// Stockham auto-sort schedule (no bit reversal): stage with radix R and
// span Ns reads R points at stride N/R, applies the twiddles
// exp(dir 2 pi i r k / (Ns R)), k = j mod Ns, performs an R-point DFT in
// registers and writes the results to (j div Ns) Ns R + k + r Ns.
//
// Three pass kinds cover a d-dimensional real transform:
//   * row R2C / C2R along x (contiguous), two real rows per complex FFT;
//   * column C2C along y or z (strided), W adjacent columns per block so
//     that every global access is a contiguous W-element segment;
//   * the last column pass fuses forward FFT, the spectral operator and the
//     inverse FFT, so the spectrum of that axis never goes back to HBM
//     between the two transforms.
#pragma once
#include <type_traits>
#include "psd_common.hpp"

namespace psd {

// ---------------------------------------------------------------------------
// radix plan: factors of 3 first, then the power of two as 16s with an 8/4/2
// tail chosen to avoid a final radix-2 stage where possible
// ---------------------------------------------------------------------------
constexpr int pow2_part(int N) { int p = 1; while (N % 2 == 0) { N /= 2; p *= 2; } return p; }
constexpr int log2i(int N) { int a = 0; while (N > 1) { N /= 2; ++a; } return a; }
constexpr int n_threes(int N) { int t = 0; while (N % 3 == 0) { N /= 3; ++t; } return t; }

constexpr int plan_stages(int N) {
  int st = n_threes(N);
  int a = log2i(pow2_part(N));
  while (a >= 4 && a != 5 && a != 6) { a -= 4; ++st; }
  if (a == 6 || a == 5) st += 2;
  else if (a > 0) st += 1;
  return st;
}

constexpr int plan_radix(int N, int s) {
  int t = n_threes(N);
  if (s < t) return 3;
  s -= t;
  int a = log2i(pow2_part(N));
  while (a >= 4 && a != 5 && a != 6) {
    if (s == 0) return 16;
    a -= 4; --s;
  }
  if (a == 6) return 8;
  if (a == 5) return s == 0 ? 8 : 4;
  if (a == 3) return 8;
  if (a == 2) return 4;
  return 2;
}

constexpr int plan_span(int N, int s) {  // product of radices of stages < s
  int p = 1;
  for (int i = 0; i < s; ++i) p *= plan_radix(N, i);
  return p;
}

// ---------------------------------------------------------------------------
// small DFTs in registers, X_q = sum_r a_r exp(DIR 2 pi i r q / R)
// ---------------------------------------------------------------------------
template <int DIR, typename T>
__device__ __forceinline__ void dft2(cx<T>& a, cx<T>& b) {
  cx<T> t = a;
  a = t + b;
  b = t - b;
}

template <int DIR, typename T>
__device__ __forceinline__ void dft4(cx<T>& a0, cx<T>& a1, cx<T>& a2, cx<T>& a3) {
  cx<T> t0 = a0 + a2, t1 = a0 - a2, t2 = a1 + a3, t3 = mul_i<DIR>(a1 - a3);
  a0 = t0 + t2;
  a2 = t0 - t2;
  a1 = t1 + t3;
  a3 = t1 - t3;
}

template <int DIR, typename T>
__device__ __forceinline__ void dft3(cx<T>* a) {
  const T c = T(0.86602540378443864676372317075293618);  // sqrt(3)/2
  cx<T> t = a[1] + a[2], d = a[1] - a[2];
  cx<T> m = a[0] - scale(t, T(0.5));
  cx<T> e = mul_i<DIR>(scale(d, c));
  a[0] = a[0] + t;
  a[1] = m + e;
  a[2] = m - e;
}

template <int DIR, typename T>
__device__ __forceinline__ void dft8(cx<T>* a) {
  const T r2 = T(0.70710678118654752440084436210484904);
  // even / odd halves
  dft4<DIR>(a[0], a[2], a[4], a[6]);
  dft4<DIR>(a[1], a[3], a[5], a[7]);
  // twiddles w^q = exp(DIR 2 pi i q / 8), q = 0..3, on the odd outputs
  cx<T> o1 = a[3], o2 = a[5], o3 = a[7];
  o1 = scale(o1 + mul_i<DIR>(o1), r2);                 // (1 + DIR i)/sqrt2
  o2 = mul_i<DIR>(o2);                                  // DIR i
  o3 = scale(mul_i<DIR>(o3) - o3, r2);                 // (-1 + DIR i)/sqrt2
  cx<T> e0 = a[0], e1 = a[2], e2 = a[4], e3 = a[6], o0 = a[1];
  a[0] = e0 + o0; a[4] = e0 - o0;
  a[1] = e1 + o1; a[5] = e1 - o1;
  a[2] = e2 + o2; a[6] = e2 - o2;
  a[3] = e3 + o3; a[7] = e3 - o3;
}

template <int DIR, typename T>
__device__ __forceinline__ void dft16(cx<T>* a) {
  // index n = 4 n1 + n2, output q = q1 + 4 q2
  const T c1 = T(0.92387953251128675612818318939678829);  // cos(pi/8)
  const T s1 = T(0.38268343236508977172845998403039887);  // sin(pi/8)
  const T r2 = T(0.70710678118654752440084436210484904);
  cx<T> y[16];
#pragma unroll
  for (int n2 = 0; n2 < 4; ++n2) {
    cx<T> b0 = a[n2], b1 = a[4 + n2], b2 = a[8 + n2], b3 = a[12 + n2];
    dft4<DIR>(b0, b1, b2, b3);
    y[n2 * 4 + 0] = b0; y[n2 * 4 + 1] = b1; y[n2 * 4 + 2] = b2; y[n2 * 4 + 3] = b3;
  }
  // twiddle y[n2][q1] *= exp(DIR 2 pi i n2 q1 / 16)
  const T ds = T(DIR);
  // n2 = 1: q1 = 1,2,3 -> angles 1,2,3 (units 2pi/16)
  y[5] = y[5] * mk(c1, ds * s1);
  y[6] = y[6] * mk(r2, ds * r2);
  y[7] = y[7] * mk(s1, ds * c1);
  // n2 = 2: angles 2,4,6
  y[9] = y[9] * mk(r2, ds * r2);
  y[10] = mul_i<DIR>(y[10]);
  y[11] = y[11] * mk(-r2, ds * r2);
  // n2 = 3: angles 3,6,9
  y[13] = y[13] * mk(s1, ds * c1);
  y[14] = y[14] * mk(-r2, ds * r2);
  y[15] = y[15] * mk(-c1, -ds * s1);
#pragma unroll
  for (int q1 = 0; q1 < 4; ++q1) {
    cx<T> b0 = y[q1], b1 = y[4 + q1], b2 = y[8 + q1], b3 = y[12 + q1];
    dft4<DIR>(b0, b1, b2, b3);
    a[q1] = b0; a[q1 + 4] = b1; a[q1 + 8] = b2; a[q1 + 12] = b3;
  }
}

template <int R, int DIR, typename T>
__device__ __forceinline__ void dftR(cx<T>* a) {
  if constexpr (R == 2) dft2<DIR>(a[0], a[1]);
  else if constexpr (R == 3) dft3<DIR>(a);
  else if constexpr (R == 4) dft4<DIR>(a[0], a[1], a[2], a[3]);
  else if constexpr (R == 8) dft8<DIR>(a);
  else dft16<DIR>(a);
}

// LDS line layout: one padding element after every 16, so that the span-1
// stage (R results per thread at stride R) does not hit the same banks from
// consecutive lanes.  Element t of a line lives at pidx(t); a line occupies
// fft_ls(N) elements.
constexpr int fft_ls(int N) { return N + N / 16 + 1; }
__device__ __forceinline__ int pidx(int t) { return t + (t >> 4); }

// Copy a table of N entries (the twiddles exp(-2 pi i m/N), m < N, or the
// fused pass's symbol) into LDS in two steps: load() issues the global loads
// into registers, store() writes them to LDS; the caller's next barrier
// publishes them.  A block issues its data loads first, then the table's,
// then stores both: the table's latency overlaps the data's instead of
// adding to it (an LDS store has to wait for its load), and the data
// requests reach memory first.
template <typename U, int N>
struct TableStage {
  static constexpr int K = (N + PSD_NT - 1) / PSD_NT;
  U v[K];
  __device__ __forceinline__ void load(const U* __restrict__ src) {
#pragma unroll
    for (int k = 0; k < K; ++k) {
      const int i = (int)threadIdx.x + k * PSD_NT;
      if (N % PSD_NT == 0 || i < N) v[k] = gld_any(src + i);
    }
    // keep the arithmetic on the block's data (which may start before the
    // next barrier) from being scheduled above these loads: it would wait
    // for the data before the table's loads are issued
    __builtin_amdgcn_sched_barrier(0);
  }
  __device__ __forceinline__ void store(U* dst) const {
#pragma unroll
    for (int k = 0; k < K; ++k) {
      const int i = (int)threadIdx.x + k * PSD_NT;
      if (N % PSD_NT == 0 || i < N) dst[i] = v[k];
    }
  }
};

template <int S, int NSTG, typename F>
__device__ __forceinline__ void stage_loop(F&& f) {
  if constexpr (S < NSTG) {
    f(std::integral_constant<int, S>());
    stage_loop<S + 1, NSTG>(f);
  }
}

// Transform NL lines of length N held in LDS (line l at buf + l*LS, element
// t at pidx(t)), in place, unnormalised: stages S0 .. S1-1 of the plan (all
// by default).  tw[m] = exp(-2 pi i m / N), staged in LDS by the caller.
// Must be called by all PSD_NT threads of the block; each stage ends with a
// barrier.
template <typename T, int N, int NL, int LS, int DIR, int S0 = 0, int S1 = plan_stages(N)>
__device__ __forceinline__ void lds_fft(cx<T>* buf, const cx<T>* __restrict__ tw) {
  stage_loop<S0, S1>([&](auto sc) {
    constexpr int s = decltype(sc)::value;
    constexpr int R = plan_radix(N, s);
    constexpr int Ns = plan_span(N, s);
    constexpr int M = N / R;             // butterflies per line
    constexpr int NB = NL * M;           // butterflies in the block
    constexpr int IT = (NB + PSD_NT - 1) / PSD_NT;
    cx<T> v[IT][R];
#pragma unroll
    for (int it = 0; it < IT; ++it) {
      const int b = threadIdx.x + it * PSD_NT;
      if (NB % PSD_NT == 0 || b < NB) {
        const int line = b / M, j = b - line * M;
        const cx<T>* src = buf + line * LS;
#pragma unroll
        for (int r = 0; r < R; ++r) v[it][r] = src[pidx(j + r * M)];
      }
    }
    __syncthreads();
#pragma unroll
    for (int it = 0; it < IT; ++it) {
      const int b = threadIdx.x + it * PSD_NT;
      if (NB % PSD_NT == 0 || b < NB) {
        const int line = b / M, j = b - line * M;
        const int k = j % Ns;
        if constexpr (Ns > 1) {
          constexpr int TS = N / (Ns * R);
#pragma unroll
          for (int r = 1; r < R; ++r) {
            cx<T> w = tw[r * k * TS];
            if (DIR > 0) w.y = -w.y;
            v[it][r] = v[it][r] * w;
          }
        }
        dftR<R, DIR>(v[it]);
        cx<T>* dst = buf + line * LS;
        const int o = (j - k) * R + k;
#pragma unroll
        for (int r = 0; r < R; ++r) dst[pidx(o + r * Ns)] = v[it][r];
      }
    }
    __syncthreads();
  });
}

// ---------------------------------------------------------------------------
// Row passes along x.  Rows are addressed globally over NF fields: row gr in
// [0, NF * rows_per_field), field = gr / rpf.  Two real rows form one complex
// line z = a + i b; after the transform A_k = (Z_k + conj Z_{N-k}) / 2 and
// B_k = -i (Z_k - conj Z_{N-k}) / 2 for k = 0..N/2.
// ---------------------------------------------------------------------------
template <typename T>
struct RowArgs {
  const void* rin0;     // real inputs per field (R2C)
  const void* rin1;
  void* rout0;          // real outputs per field (C2R)
  void* rout1;
  void* rout2;
  cx<T>* spec;          // NF fields of nspec complex
  long long nspec;      // field stride (complex elements)
  long long nyq;        // offset of the Nyquist plane (kx = N/2) in a field
  int ncp;              // row stride of the columns kx < N/2 (complex elements)
  long long rpf;        // rows per field
  long long nrows;      // rows over all fields of this pass (guard)
  // value selects (not lvalue selects), so that the struct stays in registers
  __device__ __forceinline__ const void* in(int f) const {
    const void* a = rin0;
    const void* b = rin1;
    return f == 0 ? a : b;
  }
  __device__ __forceinline__ void* out(int f) const {
    void* a = rout0;
    void* b = rout1;
    void* c = rout2;
    return f == 0 ? a : (f == 1 ? b : c);
  }
};

// Field and row of global row gr of a row pass (at most three fields of
// rpf rows each; gr < 3 rpf): comparisons instead of a 64-bit division.
__device__ __forceinline__ int row_field(long long gr, long long rpf, long long& row) {
  const int fld = (gr >= rpf ? 1 : 0) + (gr >= 2 * rpf ? 1 : 0);
  row = gr - fld * rpf;
  return fld;
}

template <typename T, typename TIN, int N, int NL>
__device__ __forceinline__ void r2c_rows(const RowArgs<T>& A, long long row0, cx<T>* buf,
                                         const cx<T>* tw) {
  constexpr int LS = fft_ls(N);
  constexpr int NC = N / 2 + 1;
  // load 2*NL real rows: VEC consecutive values per thread and load, all
  // loads of the block issued before the first LDS store
  constexpr int VEC = 16 / (int)sizeof(TIN);
  constexpr int NV = 2 * NL * N / VEC;                 // vector loads per block
  constexpr int IT = (NV + PSD_NT - 1) / PSD_NT;
  static_assert(N % VEC == 0, "row length must be a multiple of the vector width");
  struct alignas(16) V { TIN x[VEC]; };
  cx<T>* twl = buf + NL * LS;
  V regs[IT];
#pragma unroll
  for (int it = 0; it < IT; ++it) {
    const int e = threadIdx.x + it * PSD_NT;
    const int rr = (e * VEC) / N;
    const long long gr = row0 + rr;
    if ((NV % PSD_NT == 0 || e < NV) && gr < A.nrows) {
      const int col = e * VEC - rr * N;
      long long row;
      const int fld = row_field(gr, A.rpf, row);
      const gvec<TIN, VEC> g = *(const PSD_GLOBAL gvec<TIN, VEC>*)(gmem((const TIN*)A.in(fld)) + row * N + col);
#pragma unroll
      for (int q = 0; q < VEC; ++q) regs[it].x[q] = g[q];
    } else {
#pragma unroll
      for (int q = 0; q < VEC; ++q) regs[it].x[q] = TIN(0);
    }
  }
  TableStage<cx<T>, N> tws;
  tws.load(tw);
  tws.store(twl);
#pragma unroll
  for (int it = 0; it < IT; ++it) {
    const int e = threadIdx.x + it * PSD_NT;
    if (NV % PSD_NT == 0 || e < NV) {
      const int rr = (e * VEC) / N, col = e * VEC - rr * N;
      T* dst = (T*)(buf + (rr >> 1) * LS + pidx(col)) + (rr & 1);
#pragma unroll
      for (int q = 0; q < VEC; ++q) dst[2 * q] = (T)regs[it].x[q];
    }
  }
  __syncthreads();
  lds_fft<T, N, NL, LS, -1>(buf, twl);
  for (int e = threadIdx.x; e < NL * NC; e += PSD_NT) {
    const int l = e / NC, k = e - l * NC;
    const cx<T> zk = buf[l * LS + pidx(k)];
    const cx<T> zm = conj(buf[l * LS + pidx(k == 0 ? 0 : N - k)]);
    const cx<T> a = scale(zk + zm, T(0.5));
    const cx<T> b = scale(mul_i<-1>(zk - zm), T(0.5));
    const long long gr = row0 + 2 * l;
    if (gr >= A.nrows) continue;
    long long row;
    const int fld = row_field(gr, A.rpf, row);
    cx<T>* out = A.spec + fld * A.nspec;
    // rows row, row+1: columns kx < N/2 in the row array, kx = N/2 in the Nyquist plane
    const long long oa = (k < N / 2) ? row * A.ncp + k : A.nyq + row;
    const long long ob = (k < N / 2) ? oa + A.ncp : oa + 1;
    gst(out + oa, a);
    gst(out + ob, b);
  }
}

// fsum[f] accumulates the sum of the values written to output field f
template <typename T, typename TOUT, int N, int NL>
__device__ __forceinline__ void c2r_rows(const RowArgs<T>& A, long long row0, cx<T>* buf,
                                         const cx<T>* tw, double (&fsum)[3]) {
  constexpr int LS = fft_ls(N);
  constexpr int NC = N / 2 + 1;
  constexpr int NE = NL * NC;
  constexpr int IT = (NE + PSD_NT - 1) / PSD_NT;
  cx<T>* twl = buf + NL * LS;
  cx<T> ra[IT], rb[IT];
  // entries past the block's rows read its first entry, so that no branch
  // surrounds the loads (a branch splits them into separately waited
  // groups); entries past NE are not stored to LDS, and lines past the last
  // row are transformed but never written out
#pragma unroll
  for (int it = 0; it < IT; ++it) {
    const int e = threadIdx.x + it * PSD_NT;
    const int l0 = e / NC, k0 = e - l0 * NC;
    const bool ok = (NE % PSD_NT == 0 || e < NE) && row0 + 2 * l0 < A.nrows;
    const int l = ok ? l0 : 0, k = ok ? k0 : 0;
    long long row;
    const int fld = row_field(row0 + 2 * l, A.rpf, row);
    const cx<T>* in = A.spec + fld * A.nspec;
    const long long oa = (k < N / 2) ? row * A.ncp + k : A.nyq + row;
    const long long ob = (k < N / 2) ? oa + A.ncp : oa + 1;
    ra[it] = gld(in + oa);
    rb[it] = gld(in + ob);
  }
  TableStage<cx<T>, N> tws;
  tws.load(tw);
  tws.store(twl);
#pragma unroll
  for (int it = 0; it < IT; ++it) {
    const int e = threadIdx.x + it * PSD_NT;
    if (!(NE % PSD_NT == 0 || e < NE)) continue;
    const int l = e / NC, k = e - l * NC;
    cx<T> a = ra[it], b = rb[it];
    if (k == 0 || k == N / 2) { a.y = T(0); b.y = T(0); }
    // Z_k = A_k + i B_k ; Z_{N-k} = conj(A_k) + i conj(B_k)
    buf[l * LS + pidx(k)] = a + mul_i<1>(b);
    if (k != 0 && k != N / 2) buf[l * LS + pidx(N - k)] = conj(a) + mul_i<1>(conj(b));
  }
  __syncthreads();
  constexpr int SL = plan_stages(N) - 1;
  lds_fft<T, N, NL, LS, 1, 0, SL>(buf, twl);
  // The last stage of the plan (span M = N / R) keeps its results in
  // registers and writes them straight to memory: butterfly j of line l
  // holds the points j + r M (real part: row 2l, imaginary part: row 2l + 1)
  constexpr int R = plan_radix(N, SL), M = N / R, NB = NL * M;
  static_assert(plan_span(N, SL) == M, "last stage spans N / R");
  constexpr int ITL = (NB + PSD_NT - 1) / PSD_NT;
#pragma unroll
  for (int it = 0; it < ITL; ++it) {
    const int b = threadIdx.x + it * PSD_NT;
    if (!(NB % PSD_NT == 0 || b < NB)) continue;
    const int l = b / M, j = b - l * M;
    const cx<T>* src = buf + l * LS;
    cx<T> v[R];
#pragma unroll
    for (int r = 0; r < R; ++r) v[r] = src[pidx(j + r * M)];
    if constexpr (M > 1) {
#pragma unroll
      for (int r = 1; r < R; ++r) {
        cx<T> w = twl[r * j];
        w.y = -w.y;   // inverse transform: exp(+2 pi i r j / N)
        v[r] = v[r] * w;
      }
    }
    dftR<R, 1>(v);
    const long long gr = row0 + 2 * l;
    if (gr >= A.nrows) continue;
    long long row;
    const int fld = row_field(gr, A.rpf, row);
    PSD_GLOBAL TOUT* pa = gmem((TOUT*)A.out(fld)) + row * N + j;
    double part = 0.0;
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const TOUT xa = (TOUT)v[r].x, xb = (TOUT)v[r].y;
      pa[r * M] = xa;
      pa[N + r * M] = xb;
      part += (double)xa + (double)xb;
    }
    fsum[0] += fld == 0 ? part : 0.0;
    fsum[1] += fld == 1 ? part : 0.0;
    fsum[2] += fld == 2 ? part : 0.0;
  }
}

// Columns of one column-pass block: column c < ncols starts at element
// cbase + c * cstride of a field; element t of a column lies at + t * lstride
// and field f at + f * fstride.
struct ColSet {
  long long cbase, cstride, lstride;
  int ncols;
};

// Load NF fields of the block's columns of length N into LDS lines
// (f*W + c), every load of the block issued before the first LDS store;
// mid() runs between the loads and the stores (table staging).
template <typename T, int N, int W, int NF, typename Mid>
__device__ __forceinline__ void col_load(const cx<T>* base, const ColSet& cs, long long fstride,
                                         cx<T>* buf, Mid&& mid) {
  constexpr int LS = fft_ls(N);
  constexpr int NE = NF * W * N;
  constexpr int IT = (NE + PSD_NT - 1) / PSD_NT;
  static_assert(PSD_NT % W == 0, "a thread keeps one column");
  const int c = threadIdx.x % W;
  const bool live = c < cs.ncols;
  // columns past the block's last one read its first column (no branch
  // around the loads), and are zeroed afterwards
  const long long coff = cs.cbase + (live ? c : 0) * cs.cstride;
  cx<T> regs[IT];
#pragma unroll
  for (int it = 0; it < IT; ++it) {
    const int e = threadIdx.x + it * PSD_NT;
    const int ft = e / W;
    const int t = ft % N, f = ft / N;
    regs[it] = mk(T(0), T(0));
    if (NE % PSD_NT == 0 || e < NE) regs[it] = gld(base + f * fstride + coff + t * cs.lstride);
  }
  if (!live)
#pragma unroll
    for (int it = 0; it < IT; ++it) regs[it] = mk(T(0), T(0));
  mid();
#pragma unroll
  for (int it = 0; it < IT; ++it) {
    const int e = threadIdx.x + it * PSD_NT;
    if (NE % PSD_NT == 0 || e < NE) {
      const int ft = e / W;
      const int t = ft % N, f = ft / N;
      buf[(f * W + c) * LS + pidx(t)] = regs[it];
    }
  }
}

// Store NF fields of the block's columns from LDS lines (f*W + c).
template <typename T, int N, int W, int NF>
__device__ __forceinline__ void col_store(cx<T>* base, const ColSet& cs, long long fstride,
                                          const cx<T>* buf) {
  constexpr int LS = fft_ls(N);
  static_assert(PSD_NT % W == 0, "a thread keeps one column");
  const int c = threadIdx.x % W;
  if (c >= cs.ncols) return;
  const long long coff = cs.cbase + c * cs.cstride;
  for (int e = threadIdx.x; e < NF * W * N; e += PSD_NT) {
    const int ft = e / W;
    const int t = ft % N, f = ft / N;
    gst(base + f * fstride + coff + t * cs.lstride, buf[(f * W + c) * LS + pidx(t)]);
  }
}

// ---------------------------------------------------------------------------
// Column transforms with the values in registers (four-step FFT) for FP32
// lines of N = 16 N1 points, N1 = 8 or 16: W = 256 / N1 adjacent columns per
// block (W x 8 contiguous bytes per line element; W <= N/2, so a block row of
// the half spectrum fills it) and N1 threads per column.  Thread (g, c) =
// (tid / W, tid % W) holds the points g + N1 j (j < 16) of column c in x[j].
// A transform is a 16-point DFT over j, the twiddles exp(DIR 2 pi i g k / N),
// a transpose through LDS and, for each row k = g + N1 m (m < 16 / N1) the
// thread takes, an N1-point DFT across the column's threads; afterwards x[j]
// again holds output index g + N1 j.  So loads and stores of a pass use the
// same addresses whatever the direction, and a forward/inverse pair needs no
// reordering.  buf: the transpose buffer, 16 rows of FS_RS = N1 W = 256
// complex ([row][g][c]: 64-lane writes of 512 contiguous bytes).  The call
// starts with LDS writes: every thread must be past its reads of buf.
// ---------------------------------------------------------------------------
template <typename T, int N>
constexpr bool col_four_step() {
  return std::is_same<T, float>::value && PSD_NT == 256 && (N == 128 || N == 256);
}
template <int N>
constexpr int four_step_width() { return PSD_NT / (N / 16); }
constexpr int FS_RS = 256;

template <int N, int DIR, typename T>
__device__ __forceinline__ void four_step(cx<T>* x, int g, int c, cx<T>* buf, const cx<T>* twl) {
  constexpr int N1 = N / 16, W = PSD_NT / N1, M = 16 / N1;
  static_assert(N1 * W == FS_RS, "transpose buffer rows");
  dft16<DIR>(x);
#pragma unroll
  for (int k = 1; k < 16; ++k) {
    cx<T> w = twl[g * k];
    if (DIR > 0) w.y = -w.y;
    x[k] = x[k] * w;
  }
#pragma unroll
  for (int k = 0; k < 16; ++k) buf[k * FS_RS + g * W + c] = x[k];
  __syncthreads();
#pragma unroll
  for (int m = 0; m < M; ++m) {
    cx<T> v[N1];
#pragma unroll
    for (int t1 = 0; t1 < N1; ++t1) v[t1] = buf[(g + N1 * m) * FS_RS + t1 * W + c];
    dftR<N1, DIR>(v);
#pragma unroll
    for (int q = 0; q < N1; ++q) x[m + M * q] = v[q];
  }
}

// points g + N1 j of column c (zeros for a column past ncols)
template <int N, typename T>
__device__ __forceinline__ void col_fs_load(const cx<T>* base, const ColSet& cs, int c, int g, bool live,
                                            cx<T>* x) {
  // columns past the block's last one read its first column, so that the
  // loads need no branch (a branch splits them into separately waited groups)
  const cx<T>* col = base + cs.cbase + (live ? c : 0) * cs.cstride + g * cs.lstride;
  const long long step = (N / 16) * cs.lstride;
#pragma unroll
  for (int j = 0; j < 16; ++j) x[j] = gld(col + j * step);
  if (!live)
#pragma unroll
    for (int j = 0; j < 16; ++j) x[j] = mk(T(0), T(0));
}

template <int N, typename T>
__device__ __forceinline__ void col_fs_store(cx<T>* base, const ColSet& cs, int c, int g, const cx<T>* x) {
  cx<T>* col = base + cs.cbase + c * cs.cstride + g * cs.lstride;
  const long long step = (N / 16) * cs.lstride;
#pragma unroll
  for (int j = 0; j < 16; ++j) gst(col + j * step, x[j]);
}

// ---------------------------------------------------------------------------
// Column pass: the block's columns (ColSet) of length N, NF fields.  Loads,
// transforms (DIR), stores.
// ---------------------------------------------------------------------------
template <typename T, int N, int W, int NF, int DIR>
__device__ __forceinline__ void col_pass(cx<T>* base, const ColSet& cs, long long fstride, cx<T>* buf,
                                         const cx<T>* tw) {
  if constexpr (col_four_step<T, N>() && W == four_step_width<N>() && NF == 1) {
    const int c = threadIdx.x % W, g = threadIdx.x / W;
    const bool live = c < cs.ncols;
    cx<T> x[16];
    col_fs_load<N>(base, cs, c, g, live, x);
    cx<T>* twl = buf + 16 * FS_RS;
    TableStage<cx<T>, N> tws;
    tws.load(tw);
    tws.store(twl);
    __syncthreads();
    four_step<N, DIR>(x, g, c, buf, twl);
    if (live) col_fs_store<N>(base, cs, c, g, x);
    return;
  }
  constexpr int LS = fft_ls(N);
  cx<T>* twl = buf + NF * W * LS;
  TableStage<cx<T>, N> tws;
  col_load<T, N, W, NF>(base, cs, fstride, buf, [&] { tws.load(tw); tws.store(twl); });
  __syncthreads();
  lds_fft<T, N, NF * W, LS, DIR>(buf, twl);
  col_store<T, N, W, NF>(base, cs, fstride, buf);
}

}  // namespace psd
