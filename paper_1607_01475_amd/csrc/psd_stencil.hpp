// psd_stencil.hpp -- fused stencil kernels of the PSD iteration (gfx950).
//
// Discrete operators (Sec. 5.1; 3D by the same averaging construction):
//   vertex gradient   G_a(i+1/2,..) = D_a of v averaged over the 2 (2D) or
//                     4 (3D) cell pairs of the dual cell
//   divergence        div F(i,..)   = d_a of F averaged over the 2 or 4
//                     vertex pairs around the cell
//   Laplacian         Delta_h = 5-point (2D) / 7-point (3D)
//   N_h[v]            = v - s div(|G|^{p-2} G) + s eps^2 Delta_h^2 v   (Sec. 5.3)
// One kernel evaluates the residual r = f - N_h[u + alpha d] for a tile,
// writing the updated iterate to the other ping-pong buffer (the update of
// Sec. 2.2 fused with the residual of the next step), the FP64 or FP32 copy
// of r that feeds the FFT, and per-block partials of max|r| and sum r^2.
#pragma once
#include "psd_common.hpp"

namespace psd {

// tile shapes
constexpr int T2X = 64, T2Y = 8;     // 2D: 512 cells, 2 per thread
// 3D tiles: two (x,y) cell columns per thread; shapes in R3Shape / L3Shape
// 3D: planes marched per block.  The residual runs z-chunk + 2 steps, the
// line search z-chunk steps, both in groups of six: chunks with 6 | steps
// waste nothing.  Defaults and the autotuner's candidates follow that rule.
// Defaults: at 256^3 the residual's 128 tiles x 4 chunks fill its 2 blocks
// per CU, the line search's 128 tiles x 8 chunks its 4 blocks per CU.
constexpr int T3Z_RES = 64, T3Z_LS = 36;
constexpr int T3Z_MIN = 12;          // smallest chunk any tuning may pick

__device__ __forceinline__ double flux_r(double g2, double p, int p_is_4, int p_is_2) {
  if (p_is_4) return g2;
  if (p_is_2) return 1.0;
  if (p == 6.0) return g2 * g2;
  return g2 > 0.0 ? pow(g2, 0.5 * (p - 2.0)) : 0.0;
}

// Linearised flux of the second variation (Sec. 5.3) at a vertex:
//   F = |a|^{p-2} b + (p-2) |a|^{p-4} (a.b) a,  a = grad u*, b = grad xi;
// the second term is 0 where a = 0 (and for p = 2).  With I.adj_frozen set,
// the flux of the variable metric of the Remark in Sec. 3, F = |a|^{p-2} b
// (a = grad u^k, the coefficient frozen at the current iterate).
__device__ __forceinline__ void flux_lin(const Inst& I, double ax, double ay, double az, double bx,
                                         double by, double bz, double& fx, double& fy, double& fz) {
  const double a2 = ax * ax + ay * ay + az * az, ab = ax * bx + ay * by + az * bz;
  double r2, r4;
  if (I.p_is_4) { r2 = a2; r4 = 2.0; }
  else if (I.p_is_2) { r2 = 1.0; r4 = 0.0; }
  else if (I.p_is_6) { r2 = a2 * a2; r4 = 4.0 * a2; }
  else if (a2 == 0.0) { r2 = 0.0; r4 = 0.0; }
  else { r2 = pow(a2, 0.5 * (I.p - 2.0)); r4 = (I.p - 2.0) * r2 / a2; }
  if (I.adj_frozen) r4 = 0.0;
  fx = r2 * bx + r4 * ab * ax;
  fy = r2 * by + r4 * ab * ay;
  fz = r2 * bz + r4 * ab * az;
}

// ===========================================================================
// 2D residual tile (order 4 or 6)
// ===========================================================================
// LDS layout (doubles): v (TX+4)(TY+4) | lap (TX+2)(TY+2) | Fx,Fy (TX+1)(TY+1)
//                       | w (TX+2)(TY+2) (order 6)
constexpr int R2_VW = T2X + 4, R2_VH = T2Y + 4;
constexpr int R2_LW = T2X + 2, R2_LH = T2Y + 2;
constexpr int R2_FW = T2X + 1, R2_FH = T2Y + 1;
constexpr int R2_LDS = R2_VW * R2_VH + R2_LW * R2_LH + 2 * R2_FW * R2_FH + R2_LW * R2_LH;

// HESS: Hessian-vector product H xi = xi - s div(F_lin) + s eps^2 Delta_h^2 xi
// with xi = I.adj_p and u* = I.adj_us (written to I.adj_Hp; acc[1] = sum xi H xi).
// periodic 2D tile index: tiles plus halo may be wider than small grids
__device__ __forceinline__ int wrap2(int i, int n, bool small) { return small ? posmod(i, n) : wrapi(i, n); }

template <typename TD, typename TR, int ORDER, bool UPD, bool HESS = false>
__device__ void res2d_tile(const Inst& I, int x0, int y0, double* lds, double (&acc)[2]) {
  const int n = I.n;
  const bool small = n < T2X + 4;   // else every tile index lies in [-n, 2n)
  const SolveState* st = I.st;
  const int cur = st->iter & 1;
  const double alpha = UPD ? st->alpha : 0.0;
  // order 6: d, e1, e2 are mean-zero in exact arithmetic; remove the round-off mean
  const double dbar = (ORDER == 6) ? st->mean[0] : 0.0;
  const PSD_GLOBAL double* u = gmem(HESS ? (const double*)I.adj_p : (const double*)I.u[cur]);
  const PSD_GLOBAL TD* d = gmem((const TD*)I.d);
  double* v = lds;
  double* lap = v + R2_VW * R2_VH;
  double* Fx = lap + R2_LW * R2_LH;
  double* Fy = Fx + R2_FW * R2_FH;
  double* wl = Fy + R2_FW * R2_FH;
  const double ih = I.inv_h, ih2 = ih * ih;
  const int tid = threadIdx.x;

  // own cells (2 per thread): right-hand sides loaded with the tile
  constexpr int NO = T2X * T2Y / PSD_NT;
  double fo[NO], go[NO];
#pragma unroll
  for (int k = 0; k < NO; ++k) {
    const int e = tid + k * PSD_NT, ty = e / T2X, tx = e - ty * T2X;
    const long long gi = wrap2(x0 + tx, n, small) + (long long)n * wrap2(y0 + ty, n, small);
    fo[k] = HESS ? 0.0 : gmem(I.f)[gi];
    go[k] = (ORDER == 6 && !HESS) ? gmem(I.g)[gi] : 0.0;
  }
  // v = u + alpha d on the tile plus a 2-cell ring: all loads issued first,
  // with no branch around them (threads past the ring reload its last cell;
  // a branch would split the loads into separately waited groups)
  {
    constexpr int NV = R2_VW * R2_VH, IT = (NV + PSD_NT - 1) / PSD_NT;
    double uv[IT];
    TD dv[IT];
#pragma unroll
    for (int it = 0; it < IT; ++it) {
      const int e = min(tid + it * PSD_NT, NV - 1);
      const int ey = e / R2_VW, ex = e - ey * R2_VW;
      const long long gi = wrap2(x0 - 2 + ex, n, small) + (long long)n * wrap2(y0 - 2 + ey, n, small);
      uv[it] = u[gi];
      if (UPD) dv[it] = d[gi];
    }
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int it = 0; it < IT; ++it) {
      const int e = tid + it * PSD_NT;
      if (e < NV) v[e] = UPD ? uv[it] + alpha * ((double)dv[it] - dbar) : uv[it];
    }
  }
  if (HESS) {  // u* on the tile plus a 1-cell ring (vertex gradients)
    for (int e = tid; e < R2_LW * R2_LH; e += PSD_NT) {
      const int ey = e / R2_LW, ex = e - ey * R2_LW;
      const int gx = wrap2(x0 - 1 + ex, n, small), gy = wrap2(y0 - 1 + ey, n, small);
      wl[e] = gmem(I.adj_us)[gx + (long long)n * gy];
    }
  }
  if (ORDER == 6 && !HESS) {
    const double e1bar = st->mean[1], e2bar = st->mean[2];
    const PSD_GLOBAL double* w = gmem((const double*)I.w[cur]);
    const PSD_GLOBAL TD* e1 = gmem((const TD*)I.e1);
    const PSD_GLOBAL TD* e2 = gmem((const TD*)I.e2);
    constexpr int NW = R2_LW * R2_LH, IT = (NW + PSD_NT - 1) / PSD_NT;
    double wv[IT];
    TD e1v[IT], e2v[IT];
#pragma unroll
    for (int it = 0; it < IT; ++it) {
      const int e = min(tid + it * PSD_NT, NW - 1);   // as above: no branch around the loads
      const int ey = e / R2_LW, ex = e - ey * R2_LW;
      const long long gi = wrap2(x0 - 1 + ex, n, small) + (long long)n * wrap2(y0 - 1 + ey, n, small);
      wv[it] = w[gi];
      if (UPD) { e1v[it] = e1[gi]; e2v[it] = e2[gi]; }
    }
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int it = 0; it < IT; ++it) {
      const int e = tid + it * PSD_NT;
      if (e < NW)
        wl[e] = UPD ? wv[it] + (((double)e1v[it] - e1bar) - alpha * ((double)e2v[it] - e2bar)) : wv[it];
    }
  }
  __syncthreads();
  // Laplacian on the tile plus a 1-cell ring
  for (int e = tid; e < R2_LW * R2_LH; e += PSD_NT) {
    const int ly = e / R2_LW, lx = e - ly * R2_LW;
    const int c = (ly + 1) * R2_VW + lx + 1;
    lap[e] = (v[c - 1] + v[c + 1] + v[c - R2_VW] + v[c + R2_VW] - 4.0 * v[c]) * ih2;
  }
  // fluxes at vertices (i+1/2, j+1/2), i in [x0-1, x0+TX), j in [y0-1, y0+TY)
  for (int e = tid; e < R2_FW * R2_FH; e += PSD_NT) {
    const int fy = e / R2_FW, fx = e - fy * R2_FW;
    const int c = (fy + 1) * R2_VW + fx + 1;  // cell (i, j) of the vertex
    const double c00 = v[c], c10 = v[c + 1], c01 = v[c + R2_VW], c11 = v[c + R2_VW + 1];
    const double gx = 0.5 * ih * ((c10 - c00) + (c11 - c01));
    const double gy = 0.5 * ih * ((c01 - c00) + (c11 - c10));
    if (HESS) {
      const int cw = fy * R2_LW + fx;  // cell (i, j) of the vertex in the u* region
      const double s00 = wl[cw], s10 = wl[cw + 1], s01 = wl[cw + R2_LW], s11 = wl[cw + R2_LW + 1];
      const double ax = 0.5 * ih * ((s10 - s00) + (s11 - s01));
      const double ay = 0.5 * ih * ((s01 - s00) + (s11 - s10));
      double fxv, fyv, fzv;
      flux_lin(I, ax, ay, 0.0, gx, gy, 0.0, fxv, fyv, fzv);
      Fx[e] = fxv;
      Fy[e] = fyv;
    } else {
      const double rr = flux_r(gx * gx + gy * gy, I.p, I.p_is_4, I.p_is_2);
      Fx[e] = rr * gx;
      Fy[e] = rr * gy;
    }
  }
  __syncthreads();
  const double s = I.s, se2 = I.se2;
  PSD_GLOBAL double* uo = gmem(I.u[cur ^ 1]);
#pragma unroll
  for (int k = 0; k < NO; ++k) {
    const int e = tid + k * PSD_NT;
    const int ty = e / T2X, tx = e - ty * T2X;
    const int gx = x0 + tx, gy = y0 + ty;
    if (gx >= n || gy >= n) continue;
    const long long gi = gx + (long long)n * gy;
    const int fc = (ty + 1) * R2_FW + tx + 1;  // vertex (i+1/2, j+1/2)
    const double div = 0.5 * ih * ((Fx[fc] - Fx[fc - 1]) + (Fx[fc - R2_FW] - Fx[fc - R2_FW - 1]))
                     + 0.5 * ih * ((Fy[fc] - Fy[fc - R2_FW]) + (Fy[fc - 1] - Fy[fc - R2_FW - 1]));
    const int lc = (ty + 1) * R2_LW + tx + 1;
    const double l2 = (lap[lc - 1] + lap[lc + 1] + lap[lc - R2_LW] + lap[lc + R2_LW] - 4.0 * lap[lc]) * ih2;
    const double vc = v[(ty + 2) * R2_VW + tx + 2];
    if (HESS) {
      // order 4: xi - s div + s eps^2 Delta^2 xi; order 6 without its T_h part:
      // s lam xi - s div + s eps^2 Delta^2 xi
      const double hx = (ORDER == 6 ? s * I.lam : 1.0) * vc - s * div + se2 * l2;
      gmem(I.adj_Hp)[gi] = hx;
      acc[1] += vc * hx;
    } else if (ORDER == 4) {
      const double r = fo[k] - (vc - s * div + se2 * l2);
      gmem((TR*)I.r)[gi] = (TR)r;
      if (UPD) uo[gi] = vc;
      acc[0] = fmax(acc[0], fabs(r));
      acc[1] += r * r;
    } else {
      const double wc = wl[lc];
      const double lw = (wl[lc - 1] + wl[lc + 1] + wl[lc - R2_LW] + wl[lc + R2_LW] - 4.0 * wc) * ih2;
      const double r1 = go[k] - vc + lw;
      const double r2 = fo[k] - (s * I.lam * vc - s * div + se2 * l2 - wc);
      gmem((TR*)I.r1)[gi] = (TR)r1;
      gmem((TR*)I.r)[gi] = (TR)r2;
      if (UPD) { uo[gi] = vc; gmem(I.w[cur ^ 1])[gi] = wc; }
      acc[0] = fmax(acc[0], fmax(fabs(r1), fabs(r2)));
      acc[1] += r1 * r1 + r2 * r2;
    }
  }
}

// ===========================================================================
// 3D residual: a 32 x 16 column tile marching a chunk of planes in z.
// Each thread owns two (x, y) columns: their values of v = u + alpha d and of
// Delta_h v at the planes in flight stay in registers; LDS holds the xy-halo
// of 3 v planes (halo 2), 2 planes of Delta_h v (halo 1) and one vertex plane
// of fluxes stored as A = Fx + Fy, B = Fx - Fy, C = Fz, from which each
// thread forms the partial divergence of its cell for that vertex plane:
//   P = A(i,j) - A(i-1,j-1) + B(i,j-1) - B(i-1,j),  Q = sum of C over the 4
// vertices, and div = (P_below + P_above + Q_above - Q_below) / (4h).
// The global loads of planes j+3 and j+4 are in flight while plane j is
// computed.
// ===========================================================================
// Tile shape of the 3D residual: TX x (2 * 256 / TX) cell columns, two per
// thread along y.  TX = 32 (32 x 16); 64-wide tiles were measured slower at
// 256^3 (the wider halo rows cost more than the fewer single-element halo
// loads save).
constexpr int R3_CY = 2;   // cells per thread along y
template <int TX>
struct R3Shape {
  static constexpr int TY = PSD_NT / TX;        // thread rows
  static constexpr int CH = R3_CY * TY;         // cell rows of a tile
  static constexpr int VW = TX + 4, VH = CH + 4, VP = VW * VH;   // v planes (halo 2)
  static constexpr int LW = TX + 2, LH = CH + 2, LP = LW * LH;   // Laplacian planes (halo 1)
  static constexpr int FW = TX + 1, FH = CH + 1, FP = FW * FH;   // vertex planes
  static constexpr int VRING = VP - TX * CH;   // halo cells of a v plane
  static constexpr int LRING = LP - TX * CH;   // halo cells of a Laplacian plane
  static constexpr int FRING = FP - TX * CH;   // halo vertices of a flux plane
  static constexpr int LDS = 3 * VP + 2 * LP + 3 * FP;
  static constexpr int HLDS = LDS + 3 * VP;   // Hessian mode: 3 more planes (u*)
  static_assert(VRING <= PSD_NT && LRING <= PSD_NT && FRING <= PSD_NT, "ring sizes");
  // position in a v plane of halo cell number t (0 <= t < VRING)
  static __device__ __forceinline__ int vring_pos(int t) {
    if (t < 4 * VW) {                             // rows 0, 1, VH-2, VH-1
      const int r = t / VW, ex = t - r * VW;
      const int ey = r < 2 ? r : r + (VH - 4);
      return ey * VW + ex;
    }
    const int q = t - 4 * VW;                     // columns 0, 1, VW-2, VW-1 of rows 2..VH-3
    const int ey = 2 + (q >> 2), c = q & 3;
    const int ex = c < 2 ? c : c + (VW - 4);
    return ey * VW + ex;
  }
  // position in a Laplacian plane of halo cell number t (< LRING)
  static __device__ __forceinline__ int lring_pos(int t) {
    if (t < 2 * LW) {
      const int r = t / LW, lx = t - r * LW;
      return (r == 0 ? 0 : LH - 1) * LW + lx;
    }
    const int q = t - 2 * LW;
    const int ly = 1 + (q >> 1);
    return ly * LW + ((q & 1) ? LW - 1 : 0);
  }
  // position in a flux plane of halo vertex number t (< FRING)
  static __device__ __forceinline__ int fring_pos(int t) {
    if (t < FW) return t;                         // row y0-1
    return (t - FW + 1) * FW;                     // column x0-1, rows 1..FH-1
  }
};
constexpr int R3_TX = 32;

// Per-plane partial sums of the 2x2 cells (c00, c10, c01, c11) below or
// above a vertex: the vertex gradient of Sec. 5.1 (3D form) between planes k
// and k+1 is (ex_k + ex_k+1, ey_k + ey_k+1, sm_k+1 - sm_k) / (4h), so each
// plane's partials are formed once and used by the two vertex planes that
// touch it.
struct VPart {
  double ex, ey, sm;
};
__device__ __forceinline__ VPart vpart(double c00, double c10, double c01, double c11) {
  VPart q;
  q.ex = (c10 - c00) + (c11 - c01);
  q.ey = (c01 - c00) + (c11 - c10);
  q.sm = (c00 + c10) + (c01 + c11);
  return q;
}

// flux at a vertex from its two plane partials, gradients kept scaled by 4h
// (the flux is homogeneous of degree p-1; the factor (1/(4h))^p is applied
// with the divergence).  Stores A = Fx + Fy, B = Fx - Fy, C = Fz.
__device__ __forceinline__ void r3_flux(const Inst& I, const VPart& lo, const VPart& hi, double& A,
                                        double& B, double& C) {
  const double gx = lo.ex + hi.ex, gy = lo.ey + hi.ey, gz = hi.sm - lo.sm;
  const double rr = flux_r(gx * gx + gy * gy + gz * gz, I.p, I.p_is_4, I.p_is_2);
  const double fx = rr * gx, fy = rr * gy;
  A = fx + fy;
  B = fx - fy;
  C = rr * gz;
}

// HESS: linearised flux; lo/hi are partials of xi, slo/shi of u*
__device__ __forceinline__ void r3_flux_lin(const Inst& I, const VPart& lo, const VPart& hi,
                                            const VPart& slo, const VPart& shi, double& A,
                                            double& B, double& C) {
  double fx, fy, fz;
  flux_lin(I, slo.ex + shi.ex, slo.ey + shi.ey, shi.sm - slo.sm, lo.ex + hi.ex, lo.ey + hi.ey,
           hi.sm - lo.sm, fx, fy, fz);
  A = fx + fy;
  B = fx - fy;
  C = fz;
}

// flux factor |g|^{p-2} at compile-time exponent class PK (4: p = 4,
// 2: p = 2, 0: any p >= 2 at run time)
template <int PK>
__device__ __forceinline__ double flux_rr(double g2, double p) {
  if (PK == 4) return g2;
  if (PK == 2) return 1.0;
  if (PK == 6) return g2 * g2;
  return g2 > 0.0 ? pow(g2, 0.5 * (p - 2.0)) : 0.0;
}

// The plane march of a 3D residual block.  Step j (relative index
// q = j - (z0 - 2)) stores plane j+2, forms the Laplacian and the vertex
// partials of plane j+1, the fluxes of vertex plane j+1/2, and writes output
// plane j.  Every buffer rotates with period 2 or 3, so six consecutive steps
// are unrolled with compile-time buffer indices (no register copies, no
// modulo arithmetic); a block runs whole groups of six steps, steps past the
// chunk write nothing.  Thread (tx, ty) owns cells (tx, 2ty) and (tx, 2ty + 1):
// the y-neighbours inside the pair, the lower vertex of the upper cell and
// its flux come from registers (7 LDS reads for both cells' Laplacians and
// partials, 9 for their divergences, 6 for their Delta_h^2, against 10, 12
// and 8 with one cell per thread).
template <typename TD>
struct R3Prefetch {
  double u0, u1, u_ring;
  TD d0, d1, d_ring;
};

template <typename TD, typename TR, bool UPD, bool HESS, int PK, int TX>
struct Res3March {
  static constexpr bool LOADD = UPD || HESS;
  using SH = R3Shape<TX>;
  static_assert(SH::CH == 2 * SH::TY, "two cells per thread");
  static constexpr int VW = SH::VW, VP = SH::VP, LW = SH::LW, LP = SH::LP, FW = SH::FW, FP = SH::FP;
  static constexpr int VRING = SH::VRING, LRING = SH::LRING, FRING = SH::FRING;
  const Inst& I;
  const PSD_GLOBAL double* u;
  PSD_GLOBAL double* uo;
  const PSD_GLOBAL TD* d;
  const PSD_GLOBAL double* f;
  PSD_GLOBAL TR* r;
  PSD_GLOBAL double* hp;
  double* vb;   // 3 v planes
  double* lb;   // 2 Laplacian planes
  double* fA;   // one vertex plane: A, B, C
  double* fB;
  double* fC;
  double* sb;   // Hessian mode: 3 planes of u*
  double alpha, ih2, qhp, s, se2, p;
  long long nn, own0, own1, ring_xy, gout0;   // (x, y) offsets of the pair, halo cell, output
  int n, z0, z1, tid;
  // LDS positions of the pair (cell 1 = cell 0 + one row) and of this
  // thread's halo cell, halo Laplacian cell and halo vertex
  int c0, c1, l0, l1, f0, f1, vring, lring, lring_c, fring, fring_c;
  bool ok0, ok1;   // the pair's cells lie inside the grid
  // rotating registers: [plane slot][cell]
  double vc[3][2], sc[3][2], lap[3][2];
  VPart po[2][2], pr[2], so[2][2], sr[2];
  double Pq[2], Qq[2];   // per cell: divergence terms of the vertex plane below
  double fq[3][2];       // f of the output planes j, j+1, j+2: [plane slot][cell]
  R3Prefetch<TD> pf[2];
  double acc0, acc1;

  __device__ __forceinline__ Res3March(const Inst& I_, int x0, int y0, int z0_, double* lds)
      : I(I_) {
    const SolveState* st = I.st;
    const int cur = st->iter & 1;
    alpha = UPD ? st->alpha : 0.0;
    u = gmem(HESS ? (const double*)I.adj_p : (const double*)I.u[cur]);
    uo = gmem(I.u[cur ^ 1]);
    d = gmem(HESS ? (const TD*)I.adj_us : (const TD*)I.d);
    f = gmem(I.f);
    r = gmem((TR*)I.r);
    hp = gmem(I.adj_Hp);
    vb = lds;
    lb = vb + 3 * VP;
    fA = lb + 2 * LP;
    fB = fA + FP;
    fC = fB + FP;
    sb = lds + SH::LDS;
    n = I.n;
    nn = (long long)n * n;
    const double ih = I.inv_h, qh = 0.25 * ih;
    ih2 = ih * ih;
    qhp = PK == 4 ? (qh * qh) * (qh * qh)
        : (PK == 2 ? qh * qh : (PK == 6 ? (qh * qh) * (qh * qh) * (qh * qh) : pow(qh, I.p)));
    s = I.s;
    se2 = I.se2;
    p = I.p;
    z0 = z0_;
    z1 = min(z0 + I.zchunk_res, n);
    tid = threadIdx.x;
    const int tx = tid % TX, ty = tid / TX;
    c0 = (2 * ty + 2) * VW + tx + 2;
    c1 = c0 + VW;
    l0 = (2 * ty + 1) * LW + tx + 1;
    l1 = l0 + LW;
    f0 = (2 * ty + 1) * FW + tx + 1;
    f1 = f0 + FW;
    vring = tid < VRING ? SH::vring_pos(tid) : c0;
    const int rey = vring / VW, rex = vring - rey * VW;
    lring = tid < LRING ? SH::lring_pos(tid) : l0;
    lring_c = (lring / LW + 1) * VW + lring % LW + 1;
    fring = tid < FRING ? SH::fring_pos(tid) : f0;
    fring_c = (fring / FW + 1) * VW + fring % FW + 1;
    const int gx = x0 + tx, gy = y0 + 2 * ty;
    ok0 = gx < n && gy < n;
    ok1 = gx < n && gy + 1 < n;
    own0 = wrapi(gx, n) + (long long)n * wrapi(gy, n);
    own1 = wrapi(gx, n) + (long long)n * wrapi(gy + 1, n);
    ring_xy = wrapi(x0 - 2 + rex, n) + (long long)n * wrapi(y0 - 2 + rey, n);
    gout0 = gx + (long long)n * gy;
    acc0 = 0.0;
    acc1 = 0.0;
#pragma unroll
    for (int k = 0; k < 3; ++k)
#pragma unroll
      for (int e = 0; e < 2; ++e) vc[k][e] = sc[k][e] = lap[k][e] = fq[k][e] = 0.0;
#pragma unroll
    for (int k = 0; k < 2; ++k) {
      pr[k] = sr[k] = VPart{0.0, 0.0, 0.0};
#pragma unroll
      for (int e = 0; e < 2; ++e) po[k][e] = so[k][e] = VPart{0.0, 0.0, 0.0};
      Pq[k] = Qq[k] = 0.0;
    }
  }

  template <int B>
  __device__ __forceinline__ void fetch(int z) {
    const long long zo = (long long)wrapi(z, n) * nn;
    pf[B].u0 = u[zo + own0];
    pf[B].u1 = u[zo + own1];
    if (LOADD) {
      pf[B].d0 = d[zo + own0];
      pf[B].d1 = d[zo + own1];
    }
    // every thread loads a halo value (threads past the ring read a cell of
    // the tile), so that no branch surrounds the loads
    pf[B].u_ring = u[zo + ring_xy];
    if (LOADD) pf[B].d_ring = d[zo + ring_xy];
  }

  // the plane prefetched in buffer B into v slot S (and u* slot S)
  template <int S, int B>
  __device__ __forceinline__ void put() {
    const R3Prefetch<TD>& q = pf[B];
    double* vn = vb + S * VP;
    const double v0 = UPD ? q.u0 + alpha * (double)q.d0 : q.u0;
    const double v1 = UPD ? q.u1 + alpha * (double)q.d1 : q.u1;
    vn[c0] = v0;
    vn[c1] = v1;
    if (tid < VRING) vn[vring] = UPD ? q.u_ring + alpha * (double)q.d_ring : q.u_ring;
    vc[S][0] = v0;
    vc[S][1] = v1;
    if (HESS) {
      double* sn = sb + S * VP;
      sn[c0] = (double)q.d0;
      sn[c1] = (double)q.d1;
      if (tid < VRING) sn[vring] = (double)q.d_ring;
      sc[S][0] = (double)q.d0;
      sc[S][1] = (double)q.d1;
    }
  }

  __device__ __forceinline__ void flux(const VPart& lo, const VPart& hi, const VPart& slo,
                                       const VPart& shi, double& A, double& B, double& C) const {
    if (HESS) {
      r3_flux_lin(I, lo, hi, slo, shi, A, B, C);
    } else {
      const double gx = lo.ex + hi.ex, gy = lo.ey + hi.ey, gz = hi.sm - lo.sm;
      const double rr = flux_rr<PK>(gx * gx + gy * gy + gz * gz, p);
      const double fx = rr * gx, fy = rr * gy;
      A = fx + fy;
      B = fx - fy;
      C = rr * gz;
    }
  }

  __device__ __forceinline__ void prologue() {
    fetch<0>(z0 - 2);
    fetch<1>(z0 - 1);
    put<0, 0>();
    put<1, 1>();
    fetch<0>(z0);
    fetch<1>(z0 + 1);
  }

  // output value of one cell (residual, or Hessian-vector product)
  __device__ __forceinline__ void emit(long long gi, double v, double div, double l2, double fval) {
    if (HESS) {
      const double hx = v - s * div + se2 * l2;
      hp[gi] = hx;
      acc1 += v * hx;
    } else {
      const double rr = fval - (v - s * div + se2 * l2);
      // streaming stores: r and the new iterate are read again only after
      // other passes, so they are not kept in the caches, which then still
      // hold u and d for the line search and this pass
      __builtin_nontemporal_store((TR)rr, &r[gi]);
      if (UPD) __builtin_nontemporal_store(v, &uo[gi]);
      acc0 = fmax(acc0, fabs(rr));
      acc1 += rr * rr;
    }
  }

  template <int Q>
  __device__ __forceinline__ void step(int j) {
    constexpr int S0 = Q % 3, S1 = (Q + 1) % 3, S2 = (Q + 2) % 3;   // planes j, j+1, j+2
    constexpr int P0 = Q & 1, P1 = (Q + 1) & 1;                      // planes j, j+1
    // f of output plane j+2, used two steps later.  The memory counter that
    // a wait for a load tests retires loads in issue order, so f is issued
    // before the prefetch of plane j+4: the emit of plane j then waits only
    // for loads issued two steps back.  Loads are unconditional (branches
    // around them make the waits assume the worst); planes outside the
    // chunk are clamped to its last needed plane, which the caches hold.
    if (!HESS) {
      const long long fz = nn * (long long)min(j + 2, z1 - 1);
      fq[S2][0] = __builtin_nontemporal_load(&f[own0 + fz]);   // read once per iteration
      fq[S2][1] = __builtin_nontemporal_load(&f[own1 + fz]);
    }
    put<S2, P0>();
    fetch<P0>(min(j + 4, z1 + 1));
    __syncthreads();
    const double* v0 = vb + S0 * VP;
    const double* v1 = vb + S1 * VP;
    const double* v2 = vb + S2 * VP;
    // plane j+1 around the pair: x-neighbours of both cells, y- of the lower,
    // y+ and xy+ of the upper
    const double xm0 = v1[c0 - 1], xp0 = v1[c0 + 1], ym0 = v1[c0 - VW];
    const double xm1 = v1[c1 - 1], xp1 = v1[c1 + 1], yp1 = v1[c1 + VW], xyp1 = v1[c1 + VW + 1];
    double* ln = lb + P1 * LP;
    {
      const double lp0 = (xm0 + xp0 + ym0 + vc[S1][1] + vc[S0][0] + vc[S2][0] - 6.0 * vc[S1][0]) * ih2;
      const double lp1 = (xm1 + xp1 + vc[S1][0] + yp1 + vc[S0][1] + vc[S2][1] - 6.0 * vc[S1][1]) * ih2;
      ln[l0] = lp0;
      ln[l1] = lp1;
      lap[S1][0] = lp0;
      lap[S1][1] = lp1;
      if (tid < LRING) {
        const int cc = lring_c;
        ln[lring] = (v1[cc - 1] + v1[cc + 1] + v1[cc - VW] + v1[cc + VW] + v0[cc] + v2[cc] - 6.0 * v1[cc]) * ih2;
      }
    }
    // partials of plane j+1: the pair's two vertices and the ring vertex
    po[P1][0] = vpart(vc[S1][0], xp0, vc[S1][1], xp1);
    po[P1][1] = vpart(vc[S1][1], xp1, yp1, xyp1);
    pr[P1] = vpart(v1[fring_c], v1[fring_c + 1], v1[fring_c + VW], v1[fring_c + VW + 1]);
    if (HESS) {
      const double* s1 = sb + S1 * VP;
      const double sxp0 = s1[c0 + 1], sxp1 = s1[c1 + 1];
      so[P1][0] = vpart(sc[S1][0], sxp0, sc[S1][1], sxp1);
      so[P1][1] = vpart(sc[S1][1], sxp1, s1[c1 + VW], s1[c1 + VW + 1]);
      sr[P1] = vpart(s1[fring_c], s1[fring_c + 1], s1[fring_c + VW], s1[fring_c + VW + 1]);
    }
    const bool flx = j >= z0 - 1;
    double A0 = 0.0, B0 = 0.0, C0 = 0.0, A1 = 0.0, C1 = 0.0;
    if (flx) {
      double A, B, C;
      flux(po[P0][0], po[P1][0], so[P0][0], so[P1][0], A, B, C);
      fA[f0] = A; fB[f0] = B; fC[f0] = C;
      A0 = A; B0 = B; C0 = C;
      flux(po[P0][1], po[P1][1], so[P0][1], so[P1][1], A, B, C);
      fA[f1] = A; fB[f1] = B; fC[f1] = C;
      A1 = A; C1 = C;
      if (tid < FRING) {
        flux(pr[P0], pr[P1], sr[P0], sr[P1], A, B, C);
        fA[fring] = A; fB[fring] = B; fC[fring] = C;
      }
    }
    __syncthreads();
    if (flx) {
      // lower cell: vertices f0 (own), f0-1, f0-FW, f0-FW-1; upper cell: f1
      // (own), f1-1, f0 (own), f0-1
      const double fBx0 = fB[f0 - 1], fCx0 = fC[f0 - 1];
      const double P_0 = A0 - fA[f0 - FW - 1] + fB[f0 - FW] - fBx0;
      const double Q_0 = C0 + fCx0 + fC[f0 - FW] + fC[f0 - FW - 1];
      const double P_1 = A1 - fA[f0 - 1] + B0 - fB[f1 - 1];
      const double Q_1 = C1 + fC[f1 - 1] + C0 + fCx0;
      if (j >= z0 && j < z1) {
        const double* lc = lb + P0 * LP;   // Laplacian plane j
        const long long gi = gout0 + nn * j;
        if (ok0) {
          const double l2 = (lc[l0 - 1] + lc[l0 + 1] + lc[l0 - LW] + lap[S0][1] + lap[S2][0] + lap[S1][0] -
                             6.0 * lap[S0][0]) * ih2;
          emit(gi, vc[S0][0], qhp * (P_0 + Pq[0] + Q_0 - Qq[0]), l2, fq[S0][0]);
        }
        if (ok1) {
          const double l2 = (lc[l1 - 1] + lc[l1 + 1] + lap[S0][0] + lc[l1 + LW] + lap[S2][1] + lap[S1][1] -
                             6.0 * lap[S0][1]) * ih2;
          emit(gi + n, vc[S0][1], qhp * (P_1 + Pq[1] + Q_1 - Qq[1]), l2, fq[S0][1]);
        }
      }
      Pq[0] = P_0; Qq[0] = Q_0;
      Pq[1] = P_1; Qq[1] = Q_1;
    }
  }

  __device__ __forceinline__ void run() {
    prologue();
    const int T = z1 - z0 + 2;
    for (int q = 0; q < T; q += 6) {
      const int j = z0 - 2 + q;
      step<0>(j);
      step<1>(j + 1);
      step<2>(j + 2);
      step<3>(j + 3);
      step<4>(j + 4);
      step<5>(j + 5);
    }
  }
};

template <typename TD, typename TR, bool UPD, bool HESS, int PK, int TX>
__device__ __forceinline__ void res3d_tile(const Inst& I, int x0, int y0, int z0, double* lds,
                                           double (&acc)[2]) {
  static_assert(!(HESS && UPD), "no update in Hessian mode");
  static_assert(!HESS || sizeof(TD) == 8, "u* is FP64");
  Res3March<TD, TR, UPD, HESS, PK, TX> m(I, x0, y0, z0, lds);
  m.run();
  acc[0] = m.acc0;
  acc[1] = m.acc1;
}

// ===========================================================================
// 3D sixth-order residual (Sec. 5.4 mixed system, carried w) on a brick of
// B6X x B6Y x B6Z cells, everything staged in LDS:
//   v = u + alpha (d - dbar),  w' = w + (e1 - e1bar) - alpha (e2 - e2bar),
//   r1 = g - v + Delta_h w',
//   r2 = f - (s lam v - s div_h(|grad_h v|^{p-2} grad_h v) + s eps^2 Delta_h^2 v - w'),
// writing v and w' to the other ping-pong buffers, r2 and r1 (TR) for the
// FFT, and the block's max(|r1|, |r2|) and sum of r1^2 + r2^2.  HESS: the
// sixth-order Hessian without its T_h part, xi - ... replaced by
// s lam xi - s div_h(F_lin) + s eps^2 Delta_h^2 xi (the adjoint adds T_h xi).
// LDS (doubles): v (B+4)^3-brick | Laplacian (B+2) | Fx, Fy, Fz at the (B+1)
// vertices | w' (B+2) (HESS: u* there, halo 1 on the low side suffices).
// ===========================================================================
constexpr int B6X = 16, B6Y = 8, B6Z = 4;
constexpr int B6_VX = B6X + 4, B6_VY = B6Y + 4, B6_VZ = B6Z + 4, B6_V = B6_VX * B6_VY * B6_VZ;
constexpr int B6_LX = B6X + 2, B6_LY = B6Y + 2, B6_LZ = B6Z + 2, B6_L = B6_LX * B6_LY * B6_LZ;
constexpr int B6_FX = B6X + 1, B6_FY = B6Y + 1, B6_FZ = B6Z + 1, B6_F = B6_FX * B6_FY * B6_FZ;
constexpr int B6_LDS = B6_V + B6_L + 3 * B6_F + B6_L;

template <typename TD, typename TR, bool UPD, bool HESS = false>
__device__ void res3d6_tile(const Inst& I, int x0, int y0, int z0, double* lds, double (&acc)[2]) {
  const int n = I.n;
  const long long nn = (long long)n * n;
  const SolveState* st = I.st;
  const int cur = st->iter & 1;
  const double alpha = UPD ? st->alpha : 0.0;
  const double dbar = st->mean[0], e1bar = st->mean[1], e2bar = st->mean[2];
  const PSD_GLOBAL double* u = gmem(HESS ? (const double*)I.adj_p : (const double*)I.u[cur]);
  const PSD_GLOBAL TD* d = gmem((const TD*)I.d);
  double* v = lds;
  double* lap = v + B6_V;
  double* Fx = lap + B6_L;
  double* Fy = Fx + B6_F;
  double* Fz = Fy + B6_F;
  double* wl = Fz + B6_F;
  const double ih = I.inv_h, ih2 = ih * ih, q = 0.25 * ih;
  const int tid = threadIdx.x;
  auto gidx = [&](int i, int j, int k) {
    return (long long)wrapi(i, n) + (long long)n * wrapi(j, n) + nn * wrapi(k, n);
  };
  // v on the brick plus a 2-cell shell and w' (or u* in Hessian mode) on
  // the brick plus a 1-cell shell: every load is issued before the first
  // LDS store, with no branch around the loads (threads past a region
  // reload its last cell), so the block waits for memory once
  constexpr int ITV = (B6_V + PSD_NT - 1) / PSD_NT, ITW = (B6_L + PSD_NT - 1) / PSD_NT;
  constexpr bool WUPD = UPD && !HESS;
  const PSD_GLOBAL double* w = gmem(HESS ? I.adj_us : (const double*)I.w[cur]);
  const PSD_GLOBAL TD* e1 = gmem((const TD*)I.e1);
  const PSD_GLOBAL TD* e2 = gmem((const TD*)I.e2);
  double uv[ITV], wv[ITW];
  TD dv[ITV], e1v[ITW], e2v[ITW];
#pragma unroll
  for (int it = 0; it < ITV; ++it) {
    const int e = min(tid + it * PSD_NT, B6_V - 1);
    const int ex = e % B6_VX, ey = (e / B6_VX) % B6_VY, ez = e / (B6_VX * B6_VY);
    const long long gi = gidx(x0 - 2 + ex, y0 - 2 + ey, z0 - 2 + ez);
    uv[it] = u[gi];
    if (UPD) dv[it] = d[gi];
  }
#pragma unroll
  for (int it = 0; it < ITW; ++it) {
    const int e = min(tid + it * PSD_NT, B6_L - 1);
    const int ex = e % B6_LX, ey = (e / B6_LX) % B6_LY, ez = e / (B6_LX * B6_LY);
    const long long gi = gidx(x0 - 1 + ex, y0 - 1 + ey, z0 - 1 + ez);
    wv[it] = w[gi];
    if (WUPD) { e1v[it] = e1[gi]; e2v[it] = e2[gi]; }
  }
  __builtin_amdgcn_sched_barrier(0);
#pragma unroll
  for (int it = 0; it < ITV; ++it) {
    const int e = tid + it * PSD_NT;
    if (e < B6_V) v[e] = UPD ? uv[it] + alpha * ((double)dv[it] - dbar) : uv[it];
  }
#pragma unroll
  for (int it = 0; it < ITW; ++it) {
    const int e = tid + it * PSD_NT;
    if (e < B6_L) wl[e] = WUPD ? wv[it] + (((double)e1v[it] - e1bar) - alpha * ((double)e2v[it] - e2bar)) : wv[it];
  }
  __syncthreads();
  // Laplacian of v on the brick plus a 1-cell shell
  for (int e = tid; e < B6_L; e += PSD_NT) {
    const int lx = e % B6_LX, ly = (e / B6_LX) % B6_LY, lz = e / (B6_LX * B6_LY);
    const int c = (lx + 1) + B6_VX * ((ly + 1) + B6_VY * (lz + 1));
    lap[e] = (v[c - 1] + v[c + 1] + v[c - B6_VX] + v[c + B6_VX] + v[c - B6_VX * B6_VY] +
              v[c + B6_VX * B6_VY] - 6.0 * v[c]) * ih2;
  }
  // fluxes at the vertices (i+1/2, j+1/2, k+1/2), i in [x0-1, x0+B6X) etc.
  for (int e = tid; e < B6_F; e += PSD_NT) {
    const int fx = e % B6_FX, fy = (e / B6_FX) % B6_FY, fz = e / (B6_FX * B6_FY);
    const int c = (fx + 1) + B6_VX * ((fy + 1) + B6_VY * (fz + 1));   // cell (i, j, k) of the vertex
    constexpr int SY = B6_VX, SZ = B6_VX * B6_VY;
    const double c000 = v[c], c100 = v[c + 1], c010 = v[c + SY], c110 = v[c + SY + 1];
    const double c001 = v[c + SZ], c101 = v[c + SZ + 1], c011 = v[c + SZ + SY], c111 = v[c + SZ + SY + 1];
    const double gx = q * ((c100 - c000) + (c110 - c010) + (c101 - c001) + (c111 - c011));
    const double gy = q * ((c010 - c000) + (c110 - c100) + (c011 - c001) + (c111 - c101));
    const double gz = q * ((c001 - c000) + (c101 - c100) + (c011 - c010) + (c111 - c110));
    if (HESS) {
      // u* at the same 8 cells, from the shell of wl (offset 1 against v's 2)
      constexpr int TY = B6_LX, TZ = B6_LX * B6_LY;
      const int cs = fx + B6_LX * (fy + B6_LY * fz);
      const double s000 = wl[cs], s100 = wl[cs + 1], s010 = wl[cs + TY], s110 = wl[cs + TY + 1];
      const double s001 = wl[cs + TZ], s101 = wl[cs + TZ + 1], s011 = wl[cs + TZ + TY], s111 = wl[cs + TZ + TY + 1];
      const double ax = q * ((s100 - s000) + (s110 - s010) + (s101 - s001) + (s111 - s011));
      const double ay = q * ((s010 - s000) + (s110 - s100) + (s011 - s001) + (s111 - s101));
      const double az = q * ((s001 - s000) + (s101 - s100) + (s011 - s010) + (s111 - s110));
      double fxv, fyv, fzv;
      flux_lin(I, ax, ay, az, gx, gy, gz, fxv, fyv, fzv);
      Fx[e] = fxv; Fy[e] = fyv; Fz[e] = fzv;
    } else {
      const double rr = flux_r(gx * gx + gy * gy + gz * gz, I.p, I.p_is_4, I.p_is_2);
      Fx[e] = rr * gx; Fy[e] = rr * gy; Fz[e] = rr * gz;
    }
  }
  __syncthreads();
  const double s = I.s, se2 = I.se2, slam = I.s * I.lam;
  PSD_GLOBAL double* uo = gmem(I.u[cur ^ 1]);
  PSD_GLOBAL double* wo = gmem(I.w[cur ^ 1]);
  constexpr int NO = B6X * B6Y * B6Z / PSD_NT;
  for (int k = 0; k < NO; ++k) {
    const int e = tid + k * PSD_NT;
    const int tx = e % B6X, ty = (e / B6X) % B6Y, tz = e / (B6X * B6Y);
    const int gx = x0 + tx, gy = y0 + ty, gz = z0 + tz;
    if (gx >= n || gy >= n || gz >= n) continue;
    const long long gi = gx + (long long)n * gy + nn * gz;
    // vertex (i+1/2, j+1/2, k+1/2) of this cell in the flux arrays, and the 7 below / beside it
    constexpr int FY = B6_FX, FZ = B6_FX * B6_FY;
    const int f = (tx + 1) + FY * (ty + 1) + FZ * (tz + 1);
    const double divx = (Fx[f] - Fx[f - 1]) + (Fx[f - FY] - Fx[f - FY - 1]) + (Fx[f - FZ] - Fx[f - FZ - 1]) +
                        (Fx[f - FZ - FY] - Fx[f - FZ - FY - 1]);
    const double divy = (Fy[f] - Fy[f - FY]) + (Fy[f - 1] - Fy[f - FY - 1]) + (Fy[f - FZ] - Fy[f - FZ - FY]) +
                        (Fy[f - FZ - 1] - Fy[f - FZ - FY - 1]);
    const double divz = (Fz[f] - Fz[f - FZ]) + (Fz[f - 1] - Fz[f - FZ - 1]) + (Fz[f - FY] - Fz[f - FZ - FY]) +
                        (Fz[f - FY - 1] - Fz[f - FZ - FY - 1]);
    const double div = q * ((divx + divy) + divz);
    constexpr int LY = B6_LX, LZ = B6_LX * B6_LY;
    const int lc = (tx + 1) + LY * (ty + 1) + LZ * (tz + 1);
    const double l2 = (lap[lc - 1] + lap[lc + 1] + lap[lc - LY] + lap[lc + LY] + lap[lc - LZ] + lap[lc + LZ] -
                       6.0 * lap[lc]) * ih2;
    const double vc = v[(tx + 2) + B6_VX * ((ty + 2) + B6_VY * (tz + 2))];
    if (HESS) {
      const double hx = slam * vc - s * div + se2 * l2;
      gmem(I.adj_Hp)[gi] = hx;
      acc[1] += vc * hx;
      continue;
    }
    const double wc = wl[lc];
    const double lw = (wl[lc - 1] + wl[lc + 1] + wl[lc - LY] + wl[lc + LY] + wl[lc - LZ] + wl[lc + LZ] - 6.0 * wc) * ih2;
    const double r1 = gmem(I.g)[gi] - vc + lw;
    const double r2 = gmem(I.f)[gi] - (slam * vc - s * div + se2 * l2 - wc);
    gmem((TR*)I.r1)[gi] = (TR)r1;
    gmem((TR*)I.r)[gi] = (TR)r2;
    if (UPD) { uo[gi] = vc; wo[gi] = wc; }
    acc[0] = fmax(acc[0], fmax(fabs(r1), fabs(r2)));
    acc[1] += r1 * r1 + r2 * r2;
  }
}

// ===========================================================================
// Line-search sums.  MODE 0 (p = 4 cubic): S2 = sum |a|^2|b|^2,
// S3 = sum (a.b)^2, S4 = sum (a.b)|b|^2, S5 = sum |b|^4 over vertices with
// a = grad u, b = grad d; P2 = sum d^2, P4 = sum (Delta_h d)^2 over cells.
// MODE 1/2 (general p at alpha = 0 / alpha = st->x): NL = sum |g|^{p-2} g.b and
// dNL = sum |g|^{p-2}|b|^2 + (p-2)|g|^{p-4}(g.b)^2, g = a + alpha b, plus
// P2, P4.  MODE 3 (p = 6 quintic): the five vertex sums t_1 .. t_5 of
// |a + x b|^4 (a + x b).b (Sec. 6.1), plus P2, P4.  Layout of the 8 partials:
// MODE 0: S2 S3 S4 S5 P2 P4 0 0;  MODE 1/2: NL dNL P2 P4 0 0 0 0;
// MODE 3: t1 t2 t3 t4 t5 P2 P4 0.
// ===========================================================================
template <int MODE>
__device__ __forceinline__ void ls_vertex(double p, double alpha, double ax, double ay,
                                          double az, double bx, double by, double bz,
                                          double (&acc)[8]) {
  if (MODE == 0) {
    const double a2 = ax * ax + ay * ay + az * az, b2 = bx * bx + by * by + bz * bz;
    const double ab = ax * bx + ay * by + az * bz;
    acc[0] += a2 * b2;
    acc[1] += ab * ab;
    acc[2] += ab * b2;
    acc[3] += b2 * b2;
  } else if (MODE == 3) {
    // p = 6: |a + x b|^4 (a + x b).b = sum_k t_k x^k with A = |a|^2, B = a.b,
    // C = |b|^2; t_0 = A^2 B enters q(0) = -(r, d) and is not summed here
    const double A = ax * ax + ay * ay + az * az, C = bx * bx + by * by + bz * bz;
    const double B = ax * bx + ay * by + az * bz;
    const double B2 = B * B, AC = A * C;
    acc[0] += A * (AC + 4.0 * B2);           // t_1 = A^2 C + 4 A B^2
    acc[1] += B * (6.0 * AC + 4.0 * B2);     // t_2 = 6 A B C + 4 B^3
    acc[2] += C * (8.0 * B2 + 2.0 * AC);     // t_3 = 8 B^2 C + 2 A C^2
    acc[3] += 5.0 * B * C * C;               // t_4 = 5 B C^2
    acc[4] += C * C * C;                     // t_5 = C^3
  } else {
    const double gx = ax + alpha * bx, gy = ay + alpha * by, gz = az + alpha * bz;
    const double g2 = gx * gx + gy * gy + gz * gz, b2 = bx * bx + by * by + bz * bz;
    const double gb = gx * bx + gy * by + gz * bz;
    double r2, r4;
    if (p == 2.0) { r2 = 1.0; r4 = 0.0; }
    else if (g2 == 0.0) { r2 = 0.0; r4 = 0.0; }
    else { r2 = pow(g2, 0.5 * (p - 2.0)); r4 = (p - 2.0) * r2 / g2; }
    acc[0] += r2 * gb;
    acc[1] += r2 * b2 + r4 * gb * gb;
  }
}

// 2D line-search sums by rows: each wave owns 64 columns x L2W_R rows of a
// 64 x (4 L2W_R) block tile and walks its rows in order, so the rows y - 1,
// y, y + 1 a cell needs are in registers (one load per row and field), the
// x-neighbours come from the neighbouring lanes (cross-lane shuffles) and the
// halo columns x0 - 1, x0 + 64 from one extra load per row that every lane
// issues (two addresses per wave).  No LDS and no barrier until the block's
// reduction.  Each cell (x, y) contributes its vertex (x+1/2, y+1/2) (the
// averaged gradients of u and d over the 2 x 2 cells around it, Sec. 5.1)
// and its d and 5-point Laplacian of d.
constexpr int L2W_R = 8;                  // rows per wave
constexpr int L2W_X = PSD_WAVE, L2W_Y = (PSD_NT / PSD_WAVE) * L2W_R;   // block tile

template <typename TD>
struct L2wRow {
  double u, ue;       // u at the own column and at the halo column
  TD d, de;           // d likewise
};

template <typename TD, int MODE>
__device__ void ls2d_wave_tile(const Inst& I, int x0, int y0, double (&acc)[8]) {
  const int n = I.n;
  const SolveState* st = I.st;
  const PSD_GLOBAL double* u = gmem((const double*)I.u[st->iter & 1]);
  const PSD_GLOBAL TD* d = gmem((const TD*)I.d);
  const double alpha = (MODE == 2) ? st->x : 0.0;
  const int lane = threadIdx.x & (PSD_WAVE - 1), w = threadIdx.x / PSD_WAVE;
  const int ya = y0 + w * L2W_R, yb = min(ya + L2W_R, n);
  if (ya >= n) return;
  const bool okx = x0 + lane < n;
  const long long xs = posmod(x0 + lane, n);
  // halo column: x0 - 1 (lanes 0..31; lane 0 uses it), x0 + 64 (lanes 32..63; lane 63)
  const long long xe = posmod(lane < PSD_WAVE / 2 ? x0 - 1 : x0 + PSD_WAVE, n);
  const double hh = 0.5 * I.inv_h, ih2 = I.inv_h * I.inv_h;
  auto load = [&](int y, L2wRow<TD>& r) {
    const long long ro = (long long)n * wrapi(y, n);   // y in [-1, n + 1]
    r.u = u[ro + xs];
    r.ue = u[ro + xe];
    r.d = d[ro + xs];
    r.de = d[ro + xe];
  };
  auto right = [&](double v, double edge) {
    const double t = __shfl_down(v, 1, PSD_WAVE);
    return lane == PSD_WAVE - 1 ? edge : t;
  };
  auto left = [&](double v, double edge) {
    const double t = __shfl_up(v, 1, PSD_WAVE);
    return lane == 0 ? edge : t;
  };
  // row values: own, x + 1 (u and d), x - 1 (d)
  double cu, cux, cd, cdx, cdl;       // row y
  double dm = (double)d[(long long)n * wrapi(ya - 1, n) + xs];   // d at row y - 1
  L2wRow<TD> ra, rb;
  load(ya, ra);
  load(ya + 1, rb);
  cu = ra.u; cd = (double)ra.d;
  cux = right(cu, ra.ue);
  cdx = right(cd, (double)ra.de);
  cdl = left(cd, (double)ra.de);
  for (int y = ya; y < yb; ++y) {
    const L2wRow<TD> r1 = rb;
    if (y + 1 < yb) load(y + 2, rb);   // next row in flight while this one is summed
    const double nu = r1.u, nd = (double)r1.d;
    const double nux = right(nu, r1.ue);
    const double ndx = right(nd, (double)r1.de);
    const double ndl = left(nd, (double)r1.de);
    if (okx) {
      const double a00 = cu, a10 = cux, a01 = nu, a11 = nux;
      const double b00 = cd, b10 = cdx, b01 = nd, b11 = ndx;
      const double ax = hh * ((a10 - a00) + (a11 - a01)), ay = hh * ((a01 - a00) + (a11 - a10));
      const double bx = hh * ((b10 - b00) + (b11 - b01)), by = hh * ((b01 - b00) + (b11 - b10));
      ls_vertex<MODE>(I.p, alpha, ax, ay, 0.0, bx, by, 0.0, acc);
      const double ld = (cdl + cdx + dm + nd - 4.0 * b00) * ih2;
      if (MODE == 0) { acc[4] += b00 * b00; acc[5] += ld * ld; }
      else if (MODE == 3) { acc[5] += b00 * b00; acc[6] += ld * ld; }
      else { acc[2] += b00 * b00; acc[3] += ld * ld; }
    }
    dm = cd;
    cu = nu; cux = nux; cd = nd; cdx = ndx; cdl = ndl;
  }
}

// 3D line-search sums: a TX x (2 * 256/TX) column tile, two cell columns
// per thread (TX = 64 where every grid has n >= 64, else 32: wider tiles
// need fewer single-element halo loads per plane); own-column u and d in
// registers, xy-halo of 3 planes of u and d in LDS (halo 1), loads of plane
// k+2 issued before plane k is reduced.
constexpr int L3_CY = 2;   // cells per thread along y
template <int TX>
struct L3Shape {
  static constexpr int TY = PSD_NT / TX;        // thread rows
  static constexpr int CH = L3_CY * TY;         // cell rows of a tile
  static constexpr int W = TX + 2, H = CH + 2, P = W * H;
  static constexpr int RING = P - TX * CH;   // halo cells of a plane
  static constexpr int LDS = 6 * P;          // u: 3 planes, d: 3 planes
  static_assert(RING <= PSD_NT, "ring size");
  // position in a plane buffer of halo cell number t (< RING)
  static __device__ __forceinline__ int ring_pos(int t) {
    if (t < 2 * W) {
      const int r = t / W, lx = t - r * W;
      return (r == 0 ? 0 : H - 1) * W + lx;
    }
    const int q = t - 2 * W;
    const int ly = 1 + (q >> 1);
    return ly * W + ((q & 1) ? W - 1 : 0);
  }
};
constexpr int L3_TX_WIDE = 64, L3_TX_NARROW = 32;

// Thread (tx, ty) owns cells (tx, 2ty) and (tx, 2ty + 1) of the tile, so
// the lower vertex row and the Laplacian's y-neighbours come from its own
// registers: 11 LDS reads per two cells and plane instead of 18 with one
// cell per thread, and one barrier per two cells.
template <typename TD>
struct L3Prefetch {
  double u0, u1, u_ring;
  TD d0, d1, d_ring;
};

template <typename TD, int MODE, int TX>
struct Ls3March {
  using SH = L3Shape<TX>;
  static_assert(SH::CH == 2 * SH::TY, "two cells per thread");
  static constexpr int L3_W = SH::W, L3_P = SH::P, L3_RING = SH::RING;
  const Inst& I;
  const PSD_GLOBAL double* u;
  const PSD_GLOBAL TD* d;
  double* ub;
  double* db;
  double alpha, ih2;
  long long nn, own0, own1, ring_xy;
  int n, z0, z1, tid, c0, c1, ring;
  bool ok0, ok1;
  double ucol[3][2], dcol[3][2];   // own u, d of cells 0, 1 at planes (rel) r mod 3
  VPart pu[2][2], pd[2][2];        // partials of the vertices of cells 0, 1, planes r mod 2
  double n10[2][2], n01[2];        // d at x+1 of cells 0, 1 and at y+1 of cell 1, planes r mod 2
  double sacc[8];
  L3Prefetch<TD> pf;

  __device__ __forceinline__ Ls3March(const Inst& I_, int x0, int y0, int z0_, double* lds) : I(I_) {
    const SolveState* st = I.st;
    u = gmem((const double*)I.u[st->iter & 1]);
    d = gmem((const TD*)I.d);
    alpha = (MODE == 2) ? st->x : 0.0;
    ub = lds;
    db = lds + 3 * L3_P;
    ih2 = I.inv_h * I.inv_h;
    n = I.n;
    nn = (long long)n * n;
    z0 = z0_;
    z1 = min(z0 + I.zchunk_ls, n);
    tid = threadIdx.x;
    const int tx = tid % TX, ty = tid / TX;
    const int gx = x0 + tx, gy = y0 + 2 * ty;
    ok0 = gx < n && gy < n;
    ok1 = gx < n && gy + 1 < n;
    c0 = (2 * ty + 1) * L3_W + tx + 1;
    c1 = c0 + L3_W;
    ring = tid < L3_RING ? SH::ring_pos(tid) : c0;
    const int rey = ring / L3_W, rex = ring - rey * L3_W;
    own0 = wrapi(gx, n) + (long long)n * wrapi(gy, n);
    own1 = wrapi(gx, n) + (long long)n * wrapi(gy + 1, n);
    ring_xy = tid < L3_RING ? wrapi(x0 - 1 + rex, n) + (long long)n * wrapi(y0 - 1 + rey, n) : own0;
#pragma unroll
    for (int k = 0; k < 3; ++k) ucol[k][0] = ucol[k][1] = dcol[k][0] = dcol[k][1] = 0.0;
#pragma unroll
    for (int k = 0; k < 2; ++k) {
      pu[k][0] = pu[k][1] = pd[k][0] = pd[k][1] = VPart{0.0, 0.0, 0.0};
      n10[k][0] = n10[k][1] = n01[k] = 0.0;
    }
#pragma unroll
    for (int k = 0; k < 8; ++k) sacc[k] = 0.0;
  }

  __device__ __forceinline__ void fetch(int z) {
    const long long zo = (long long)wrapi(z, n) * nn;
    pf.u0 = u[zo + own0];
    pf.u1 = u[zo + own1];
    pf.d0 = d[zo + own0];
    pf.d1 = d[zo + own1];
    if (tid < L3_RING) {
      pf.u_ring = u[zo + ring_xy];
      pf.d_ring = d[zo + ring_xy];
    }
  }

  template <int S>
  __device__ __forceinline__ void put() {
    double* us = ub + S * L3_P;
    double* ds = db + S * L3_P;
    us[c0] = pf.u0;
    us[c1] = pf.u1;
    ds[c0] = (double)pf.d0;
    ds[c1] = (double)pf.d1;
    if (tid < L3_RING) {
      us[ring] = pf.u_ring;
      ds[ring] = (double)pf.d_ring;
    }
    ucol[S][0] = pf.u0;
    ucol[S][1] = pf.u1;
    dcol[S][0] = (double)pf.d0;
    dcol[S][1] = (double)pf.d1;
  }

  // partials of the plane in slot S into register slot R
  template <int S, int R>
  __device__ __forceinline__ void partials() {
    const double* u1 = ub + S * L3_P;
    const double* d1 = db + S * L3_P;
    const double ua = u1[c0 + 1], ub1 = u1[c1 + 1], uc = u1[c1 + L3_W], ud = u1[c1 + L3_W + 1];
    pu[R][0] = vpart(ucol[S][0], ua, ucol[S][1], ub1);
    pu[R][1] = vpart(ucol[S][1], ub1, uc, ud);
    const double da = d1[c0 + 1], db1 = d1[c1 + 1], dc = d1[c1 + L3_W], dd = d1[c1 + L3_W + 1];
    pd[R][0] = vpart(dcol[S][0], da, dcol[S][1], db1);
    pd[R][1] = vpart(dcol[S][1], db1, dc, dd);
    n10[R][0] = da;
    n10[R][1] = db1;
    n01[R] = dc;
  }

  __device__ __forceinline__ void vertex(const VPart& a0, const VPart& a1, const VPart& b0, const VPart& b1) {
    const double ax = a0.ex + a1.ex, ay = a0.ey + a1.ey, az = a1.sm - a0.sm;
    const double bx = b0.ex + b1.ex, by = b0.ey + b1.ey, bz = b1.sm - b0.sm;
    ls_vertex<MODE>(I.p, alpha, ax, ay, az, bx, by, bz, sacc);
  }

  __device__ __forceinline__ void cell(double dk, double ld) {
    if (MODE == 0) { sacc[4] += dk * dk; sacc[5] += ld * ld; }
    else if (MODE == 3) { sacc[5] += dk * dk; sacc[6] += ld * ld; }
    else { sacc[2] += dk * dk; sacc[3] += ld * ld; }
  }

  // plane z0-1 enters only through the own d; plane z0 in slot 1; plane
  // z0+1 in flight
  __device__ __forceinline__ void prologue() {
    const long long zm = (long long)wrapi(z0 - 1, n) * nn;
    dcol[0][0] = (double)d[zm + own0];
    dcol[0][1] = (double)d[zm + own1];
    fetch(z0);
    put<1>();
    fetch(z0 + 1);
    __syncthreads();
    partials<1, 1>();
  }

  template <int Q>
  __device__ __forceinline__ void step(int k) {
    // relative plane index r = plane - z0 + 1: k-1 -> q, k -> q+1, k+1 -> q+2
    constexpr int SM = Q % 3, SK = (Q + 1) % 3, SN = (Q + 2) % 3;
    constexpr int RK = (Q + 1) & 1, RN = Q & 1;
    put<SN>();
    fetch(k + 2);   // planes past the chunk are read and never used
    __syncthreads();
    partials<SN, RN>();
    if (k < z1) {
      const double* d0 = db + SK * L3_P;
      if (ok0) {
        vertex(pu[RK][0], pu[RN][0], pd[RK][0], pd[RN][0]);
        const double dk = dcol[SK][0];
        cell(dk, (d0[c0 - 1] + n10[RK][0] + d0[c0 - L3_W] + dcol[SK][1] + dcol[SM][0] + dcol[SN][0] -
                  6.0 * dk) * ih2);
      }
      if (ok1) {
        vertex(pu[RK][1], pu[RN][1], pd[RK][1], pd[RN][1]);
        const double dk = dcol[SK][1];
        cell(dk, (d0[c1 - 1] + n10[RK][1] + dcol[SK][0] + n01[RK] + dcol[SM][1] + dcol[SN][1] -
                  6.0 * dk) * ih2);
      }
    }
  }

  __device__ __forceinline__ void run() {
    prologue();
    const int T = z1 - z0;
    for (int q = 0; q < T; q += 6) {
      const int k = z0 + q;
      step<0>(k);
      step<1>(k + 1);
      step<2>(k + 2);
      step<3>(k + 3);
      step<4>(k + 4);
      step<5>(k + 5);
    }
  }
};

template <typename TD, int MODE, int TX>
__device__ __forceinline__ void ls3d_tile(const Inst& I, int x0, int y0, int z0, double* lds,
                                          double (&acc)[8]) {
  Ls3March<TD, MODE, TX> m(I, x0, y0, z0, lds);
  m.run();
  // vertex sums were taken with gradients scaled by 4h: undo once
  const double qh = 0.25 * I.inv_h, qh2 = qh * qh;
  const double sc = (MODE == 0 || I.p_is_4) ? qh2 * qh2
                  : ((MODE == 3 || I.p_is_6) ? qh2 * qh2 * qh2 : pow(qh, I.p));
  if (MODE == 0) {
    for (int q = 0; q < 4; ++q) acc[q] += sc * m.sacc[q];
    acc[4] += m.sacc[4]; acc[5] += m.sacc[5];
  } else if (MODE == 3) {
    for (int q = 0; q < 5; ++q) acc[q] += sc * m.sacc[q];
    acc[5] += m.sacc[5]; acc[6] += m.sacc[6];
  } else {
    acc[0] += sc * m.sacc[0]; acc[1] += sc * m.sacc[1];
    acc[2] += m.sacc[2]; acc[3] += m.sacc[3];
  }
}

}  // namespace psd
