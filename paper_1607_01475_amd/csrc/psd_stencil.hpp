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
constexpr int T3X = 32, T3Y = 8;     // 3D: one (x,y) column per thread
constexpr int T3Z = 16;              // 3D: planes marched per block

__device__ __forceinline__ double flux_r(double g2, double p, int p_is_4, int p_is_2) {
  if (p_is_4) return g2;
  if (p_is_2) return 1.0;
  return g2 > 0.0 ? pow(g2, 0.5 * (p - 2.0)) : 0.0;
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

template <typename TD, typename TR, int ORDER, bool UPD>
__device__ void res2d_tile(const Inst& I, int x0, int y0, double* lds, double (&acc)[2]) {
  const int n = I.n;
  const SolveState* st = I.st;
  const int cur = st->iter & 1;
  const double alpha = UPD ? st->alpha : 0.0;
  // order 6: d, e1, e2 are mean-zero in exact arithmetic; remove the round-off mean
  const double dbar = (ORDER == 6) ? st->mean[0] : 0.0;
  const double* __restrict__ u = I.u[cur];
  const TD* __restrict__ d = (const TD*)I.d;
  double* v = lds;
  double* lap = v + R2_VW * R2_VH;
  double* Fx = lap + R2_LW * R2_LH;
  double* Fy = Fx + R2_FW * R2_FH;
  double* wl = Fy + R2_FW * R2_FH;
  const double ih = I.inv_h, ih2 = ih * ih;

  for (int e = threadIdx.x; e < R2_VW * R2_VH; e += PSD_NT) {
    const int ey = e / R2_VW, ex = e - ey * R2_VW;
    const int gx = posmod(x0 - 2 + ex, n), gy = posmod(y0 - 2 + ey, n);
    const long long gi = gx + (long long)n * gy;
    double val = u[gi];
    if (UPD) val += alpha * ((double)d[gi] - dbar);
    v[e] = val;
  }
  if (ORDER == 6) {
    const double e1bar = st->mean[1], e2bar = st->mean[2];
    const double* __restrict__ w = I.w[cur];
    const TD* __restrict__ e1 = (const TD*)I.e1;
    const TD* __restrict__ e2 = (const TD*)I.e2;
    for (int e = threadIdx.x; e < R2_LW * R2_LH; e += PSD_NT) {
      const int ey = e / R2_LW, ex = e - ey * R2_LW;
      const int gx = posmod(x0 - 1 + ex, n), gy = posmod(y0 - 1 + ey, n);
      const long long gi = gx + (long long)n * gy;
      double val = w[gi];
      if (UPD) val += ((double)e1[gi] - e1bar) - alpha * ((double)e2[gi] - e2bar);
      wl[e] = val;
    }
  }
  __syncthreads();
  // Laplacian on the tile plus a 1-cell ring
  for (int e = threadIdx.x; e < R2_LW * R2_LH; e += PSD_NT) {
    const int ly = e / R2_LW, lx = e - ly * R2_LW;
    const int c = (ly + 1) * R2_VW + lx + 1;
    lap[e] = (v[c - 1] + v[c + 1] + v[c - R2_VW] + v[c + R2_VW] - 4.0 * v[c]) * ih2;
  }
  // fluxes at vertices (i+1/2, j+1/2), i in [x0-1, x0+TX), j in [y0-1, y0+TY)
  for (int e = threadIdx.x; e < R2_FW * R2_FH; e += PSD_NT) {
    const int fy = e / R2_FW, fx = e - fy * R2_FW;
    const int c = (fy + 1) * R2_VW + fx + 1;  // cell (i, j) of the vertex
    const double c00 = v[c], c10 = v[c + 1], c01 = v[c + R2_VW], c11 = v[c + R2_VW + 1];
    const double gx = 0.5 * ih * ((c10 - c00) + (c11 - c01));
    const double gy = 0.5 * ih * ((c01 - c00) + (c11 - c10));
    const double rr = flux_r(gx * gx + gy * gy, I.p, I.p_is_4, I.p_is_2);
    Fx[e] = rr * gx;
    Fy[e] = rr * gy;
  }
  __syncthreads();
  const double s = I.s, se2 = I.se2;
  double* __restrict__ uo = I.u[cur ^ 1];
  for (int e = threadIdx.x; e < T2X * T2Y; e += PSD_NT) {
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
    if (ORDER == 4) {
      const double r = I.f[gi] - (vc - s * div + se2 * l2);
      ((TR*)I.r)[gi] = (TR)r;
      if (UPD) uo[gi] = vc;
      acc[0] = fmax(acc[0], fabs(r));
      acc[1] += r * r;
    } else {
      const double wc = wl[lc];
      const double lw = (wl[lc - 1] + wl[lc + 1] + wl[lc - R2_LW] + wl[lc + R2_LW] - 4.0 * wc) * ih2;
      const double r1 = I.g[gi] - vc + lw;
      const double r2 = I.f[gi] - (s * I.lam * vc - s * div + se2 * l2 - wc);
      ((TR*)I.r1)[gi] = (TR)r1;
      ((TR*)I.r)[gi] = (TR)r2;
      if (UPD) { uo[gi] = vc; I.w[cur ^ 1][gi] = wc; }
      acc[0] = fmax(acc[0], fmax(fabs(r1), fabs(r2)));
      acc[1] += r1 * r1 + r2 * r2;
    }
  }
}

// ===========================================================================
// 3D residual: (T3X x T3Y) column tile marching T3Z planes in z.
// Ring buffers: v 4 planes (halo 2), lap 3 planes (halo 1), F 2 vertex planes.
// ===========================================================================
constexpr int R3_VW = T3X + 4, R3_VH = T3Y + 4, R3_VP = R3_VW * R3_VH;
constexpr int R3_LW = T3X + 2, R3_LH = T3Y + 2, R3_LP = R3_LW * R3_LH;
constexpr int R3_FW = T3X + 1, R3_FH = T3Y + 1, R3_FP = R3_FW * R3_FH;
constexpr int R3_LDS = 4 * R3_VP + 3 * R3_LP + 2 * 3 * R3_FP;

template <typename TD, bool UPD>
__device__ __forceinline__ void r3_load_plane(const Inst& I, const double* __restrict__ u,
                                              const TD* __restrict__ d, double alpha, int x0, int y0,
                                              int z, double* vp) {
  const int n = I.n;
  const long long zo = (long long)wrapi(z, n) * n * n;
  for (int e = threadIdx.x; e < R3_VP; e += PSD_NT) {
    const int ey = e / R3_VW, ex = e - ey * R3_VW;
    const int gx = wrapi(x0 - 2 + ex, n), gy = wrapi(y0 - 2 + ey, n);
    const long long gi = zo + gx + (long long)n * gy;
    double val = u[gi];
    if (UPD) val += alpha * (double)d[gi];
    vp[e] = val;
  }
}

__device__ __forceinline__ void r3_lap_plane(const double* vm, const double* v0, const double* vp,
                                             double* lp, double ih2) {
  for (int e = threadIdx.x; e < R3_LP; e += PSD_NT) {
    const int ly = e / R3_LW, lx = e - ly * R3_LW;
    const int c = (ly + 1) * R3_VW + lx + 1;
    lp[e] = (v0[c - 1] + v0[c + 1] + v0[c - R3_VW] + v0[c + R3_VW] + vm[c] + vp[c] - 6.0 * v0[c]) * ih2;
  }
}

// fluxes at vertex plane between cell planes v0 (lower) and v1 (upper)
__device__ __forceinline__ void r3_flux_plane(const Inst& I, const double* v0, const double* v1,
                                              double* F, double qh) {
  for (int e = threadIdx.x; e < R3_FP; e += PSD_NT) {
    const int fy = e / R3_FW, fx = e - fy * R3_FW;
    const int c = (fy + 1) * R3_VW + fx + 1;
    const double c000 = v0[c], c100 = v0[c + 1], c010 = v0[c + R3_VW], c110 = v0[c + R3_VW + 1];
    const double c001 = v1[c], c101 = v1[c + 1], c011 = v1[c + R3_VW], c111 = v1[c + R3_VW + 1];
    const double gx = qh * ((c100 - c000) + (c110 - c010) + (c101 - c001) + (c111 - c011));
    const double gy = qh * ((c010 - c000) + (c110 - c100) + (c011 - c001) + (c111 - c101));
    const double gz = qh * ((c001 - c000) + (c101 - c100) + (c011 - c010) + (c111 - c110));
    const double rr = flux_r(gx * gx + gy * gy + gz * gz, I.p, I.p_is_4, I.p_is_2);
    F[e] = rr * gx;
    F[R3_FP + e] = rr * gy;
    F[2 * R3_FP + e] = rr * gz;
  }
}

template <typename TD, typename TR, bool UPD>
__device__ void res3d_tile(const Inst& I, int x0, int y0, int z0, double* lds, double (&acc)[2]) {
  const int n = I.n;
  const SolveState* st = I.st;
  const int cur = st->iter & 1;
  const double alpha = UPD ? st->alpha : 0.0;
  const double* __restrict__ u = I.u[cur];
  double* __restrict__ uo = I.u[cur ^ 1];
  const TD* __restrict__ d = (const TD*)I.d;
  double* vb = lds;                    // 4 planes
  double* lb = vb + 4 * R3_VP;         // 3 planes
  double* fb = lb + 3 * R3_LP;         // 2 vertex planes x 3 components
  const double ih = I.inv_h, ih2 = ih * ih, qh = 0.25 * ih;
  const double s = I.s, se2 = I.se2;
  const int z1 = min(z0 + T3Z, n);
  // prologue: v planes z0-2 .. z0+1, lap z0-1, z0, flux plane z0-1
  for (int q = -2; q <= 1; ++q) r3_load_plane<TD, UPD>(I, u, d, alpha, x0, y0, z0 + q, vb + ((z0 + q + 8) & 3) * R3_VP);
  __syncthreads();
  for (int q = -1; q <= 0; ++q)
    r3_lap_plane(vb + ((z0 + q - 1 + 8) & 3) * R3_VP, vb + ((z0 + q + 8) & 3) * R3_VP,
                 vb + ((z0 + q + 1 + 8) & 3) * R3_VP, lb + ((z0 + q + 3) % 3) * R3_LP, ih2);
  r3_flux_plane(I, vb + ((z0 - 1 + 8) & 3) * R3_VP, vb + ((z0 + 8) & 3) * R3_VP,
                fb + ((z0 - 1 + 2) & 1) * 3 * R3_FP, qh);
  __syncthreads();  // the first in-loop load reuses the slot of plane z0-2
  const int tx = threadIdx.x % T3X, ty = threadIdx.x / T3X;
  const int gx = x0 + tx, gy = y0 + ty;
  const bool own = gx < n && gy < n;
  for (int k = z0; k < z1; ++k) {
    r3_load_plane<TD, UPD>(I, u, d, alpha, x0, y0, k + 2, vb + ((k + 2) & 3) * R3_VP);
    __syncthreads();
    r3_lap_plane(vb + (k & 3) * R3_VP, vb + ((k + 1) & 3) * R3_VP, vb + ((k + 2) & 3) * R3_VP,
                 lb + ((k + 1) % 3) * R3_LP, ih2);
    r3_flux_plane(I, vb + (k & 3) * R3_VP, vb + ((k + 1) & 3) * R3_VP, fb + ((k + 2) & 1) * 3 * R3_FP, qh);
    __syncthreads();
    if (own) {
      const double* F0 = fb + ((k + 1) & 1) * 3 * R3_FP;  // vertex plane k-1/2
      const double* F1 = fb + ((k + 2) & 1) * 3 * R3_FP;  // vertex plane k+1/2
      const int fc = (ty + 1) * R3_FW + tx + 1;
      const int fx = fc - 1, fy = fc - R3_FW, fxy = fc - R3_FW - 1;
      const double* Fx0 = F0; const double* Fy0 = F0 + R3_FP; const double* Fz0 = F0 + 2 * R3_FP;
      const double* Fx1 = F1; const double* Fy1 = F1 + R3_FP; const double* Fz1 = F1 + 2 * R3_FP;
      const double dx = (Fx1[fc] - Fx1[fx]) + (Fx1[fy] - Fx1[fxy]) + (Fx0[fc] - Fx0[fx]) + (Fx0[fy] - Fx0[fxy]);
      const double dy = (Fy1[fc] - Fy1[fy]) + (Fy1[fx] - Fy1[fxy]) + (Fy0[fc] - Fy0[fy]) + (Fy0[fx] - Fy0[fxy]);
      const double dz = (Fz1[fc] - Fz0[fc]) + (Fz1[fx] - Fz0[fx]) + (Fz1[fy] - Fz0[fy]) + (Fz1[fxy] - Fz0[fxy]);
      const double div = qh * (dx + dy + dz);
      const double* lm = lb + ((k + 2) % 3) * R3_LP;  // plane k-1
      const double* l0 = lb + (k % 3) * R3_LP;
      const double* lp = lb + ((k + 1) % 3) * R3_LP;
      const int lc = (ty + 1) * R3_LW + tx + 1;
      const double l2 = (l0[lc - 1] + l0[lc + 1] + l0[lc - R3_LW] + l0[lc + R3_LW] + lm[lc] + lp[lc] - 6.0 * l0[lc]) * ih2;
      const double vc = vb[(k & 3) * R3_VP + (ty + 2) * R3_VW + tx + 2];
      const long long gi = gx + (long long)n * (gy + (long long)n * k);
      const double r = I.f[gi] - (vc - s * div + se2 * l2);
      ((TR*)I.r)[gi] = (TR)r;
      if (UPD) uo[gi] = vc;
      acc[0] = fmax(acc[0], fabs(r));
      acc[1] += r * r;
    }
  }
}

// ===========================================================================
// Line-search sums.  MODE 0 (p = 4 cubic): S2 = sum |a|^2|b|^2,
// S3 = sum (a.b)^2, S4 = sum (a.b)|b|^2, S5 = sum |b|^4 over vertices with
// a = grad u, b = grad d; P2 = sum d^2, P4 = sum (Delta_h d)^2 over cells.
// MODE 1/2 (general p at alpha = 0 / alpha = st->x): NL = sum |g|^{p-2} g.b and
// dNL = sum |g|^{p-2}|b|^2 + (p-2)|g|^{p-4}(g.b)^2, g = a + alpha b, plus
// P2, P4.  Layout of the 8 partials: MODE 0: S2 S3 S4 S5 P2 P4 0 0;
// MODE 1: NL dNL P2 P4 0 0 0 0.
// ===========================================================================
__device__ __forceinline__ void ls_vertex(int mode, double p, double alpha, double ax, double ay,
                                          double az, double bx, double by, double bz,
                                          double (&acc)[8]) {
  if (mode == 0) {
    const double a2 = ax * ax + ay * ay + az * az, b2 = bx * bx + by * by + bz * bz;
    const double ab = ax * bx + ay * by + az * bz;
    acc[0] += a2 * b2;
    acc[1] += ab * ab;
    acc[2] += ab * b2;
    acc[3] += b2 * b2;
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

constexpr int L2_W = T2X + 2, L2_H = T2Y + 2;
constexpr int L2_LDS = 2 * L2_W * L2_H;

template <typename TD>
__device__ void ls2d_tile(const Inst& I, int mode, int x0, int y0, double* lds, double (&acc)[8]) {
  const int n = I.n;
  const SolveState* st = I.st;
  const double* __restrict__ u = I.u[st->iter & 1];
  const TD* __restrict__ d = (const TD*)I.d;
  const double alpha = (mode == 2) ? st->x : 0.0;
  double* ul = lds;
  double* dl = lds + L2_W * L2_H;
  for (int e = threadIdx.x; e < L2_W * L2_H; e += PSD_NT) {
    const int ey = e / L2_W, ex = e - ey * L2_W;
    const int gx = posmod(x0 - 1 + ex, n), gy = posmod(y0 - 1 + ey, n);
    const long long gi = gx + (long long)n * gy;
    ul[e] = u[gi];
    dl[e] = (double)d[gi];
  }
  __syncthreads();
  const double hh = 0.5 * I.inv_h, ih2 = I.inv_h * I.inv_h;
  for (int e = threadIdx.x; e < T2X * T2Y; e += PSD_NT) {
    const int ty = e / T2X, tx = e - ty * T2X;
    if (x0 + tx >= n || y0 + ty >= n) continue;
    const int c = (ty + 1) * L2_W + tx + 1;
    const double a00 = ul[c], a10 = ul[c + 1], a01 = ul[c + L2_W], a11 = ul[c + L2_W + 1];
    const double b00 = dl[c], b10 = dl[c + 1], b01 = dl[c + L2_W], b11 = dl[c + L2_W + 1];
    const double ax = hh * ((a10 - a00) + (a11 - a01)), ay = hh * ((a01 - a00) + (a11 - a10));
    const double bx = hh * ((b10 - b00) + (b11 - b01)), by = hh * ((b01 - b00) + (b11 - b10));
    ls_vertex(mode, I.p, alpha, ax, ay, 0.0, bx, by, 0.0, acc);
    const double ld = (dl[c - 1] + dl[c + 1] + dl[c - L2_W] + dl[c + L2_W] - 4.0 * b00) * ih2;
    if (mode == 0) { acc[4] += b00 * b00; acc[5] += ld * ld; }
    else { acc[2] += b00 * b00; acc[3] += ld * ld; }
  }
}

constexpr int L3_W = T3X + 2, L3_H = T3Y + 2, L3_P = L3_W * L3_H;
constexpr int L3_LDS = 6 * L3_P;  // u: 3 planes, d: 3 planes

template <typename TD>
__device__ __forceinline__ void l3_load(const Inst& I, const double* __restrict__ u,
                                        const TD* __restrict__ d, int x0, int y0, int z,
                                        double* up, double* dp) {
  const int n = I.n;
  const long long zo = (long long)wrapi(z, n) * n * n;
  for (int e = threadIdx.x; e < L3_P; e += PSD_NT) {
    const int ey = e / L3_W, ex = e - ey * L3_W;
    const int gx = wrapi(x0 - 1 + ex, n), gy = wrapi(y0 - 1 + ey, n);
    const long long gi = zo + gx + (long long)n * gy;
    up[e] = u[gi];
    dp[e] = (double)d[gi];
  }
}

template <typename TD>
__device__ void ls3d_tile(const Inst& I, int mode, int x0, int y0, int z0, double* lds,
                          double (&acc)[8]) {
  const int n = I.n;
  const SolveState* st = I.st;
  const double* __restrict__ u = I.u[st->iter & 1];
  const TD* __restrict__ d = (const TD*)I.d;
  const double alpha = (mode == 2) ? st->x : 0.0;
  double* ub = lds;
  double* db = lds + 3 * L3_P;
  const double qh = 0.25 * I.inv_h, ih2 = I.inv_h * I.inv_h;
  const int z1 = min(z0 + T3Z, n);
  l3_load<TD>(I, u, d, x0, y0, z0 - 1, ub + ((z0 + 2) % 3) * L3_P, db + ((z0 + 2) % 3) * L3_P);
  l3_load<TD>(I, u, d, x0, y0, z0, ub + (z0 % 3) * L3_P, db + (z0 % 3) * L3_P);
  const int tx = threadIdx.x % T3X, ty = threadIdx.x / T3X;
  const bool own = x0 + tx < n && y0 + ty < n;
  const int c = (ty + 1) * L3_W + tx + 1;
  for (int k = z0; k < z1; ++k) {
    l3_load<TD>(I, u, d, x0, y0, k + 1, ub + ((k + 1) % 3) * L3_P, db + ((k + 1) % 3) * L3_P);
    __syncthreads();
    if (own) {
      const double* u0 = ub + (k % 3) * L3_P;
      const double* u1 = ub + ((k + 1) % 3) * L3_P;
      const double* d0 = db + (k % 3) * L3_P;
      const double* d1 = db + ((k + 1) % 3) * L3_P;
      const double* dm = db + ((k + 2) % 3) * L3_P;
      const double a000 = u0[c], a100 = u0[c + 1], a010 = u0[c + L3_W], a110 = u0[c + L3_W + 1];
      const double a001 = u1[c], a101 = u1[c + 1], a011 = u1[c + L3_W], a111 = u1[c + L3_W + 1];
      const double b000 = d0[c], b100 = d0[c + 1], b010 = d0[c + L3_W], b110 = d0[c + L3_W + 1];
      const double b001 = d1[c], b101 = d1[c + 1], b011 = d1[c + L3_W], b111 = d1[c + L3_W + 1];
      const double ax = qh * ((a100 - a000) + (a110 - a010) + (a101 - a001) + (a111 - a011));
      const double ay = qh * ((a010 - a000) + (a110 - a100) + (a011 - a001) + (a111 - a101));
      const double az = qh * ((a001 - a000) + (a101 - a100) + (a011 - a010) + (a111 - a110));
      const double bx = qh * ((b100 - b000) + (b110 - b010) + (b101 - b001) + (b111 - b011));
      const double by = qh * ((b010 - b000) + (b110 - b100) + (b011 - b001) + (b111 - b101));
      const double bz = qh * ((b001 - b000) + (b101 - b100) + (b011 - b010) + (b111 - b110));
      ls_vertex(mode, I.p, alpha, ax, ay, az, bx, by, bz, acc);
      const double ld = (d0[c - 1] + d0[c + 1] + d0[c - L3_W] + d0[c + L3_W] + dm[c] + d1[c] - 6.0 * b000) * ih2;
      if (mode == 0) { acc[4] += b000 * b000; acc[5] += ld * ld; }
      else { acc[2] += b000 * b000; acc[3] += ld * ld; }
    }
    __syncthreads();
  }
}

}  // namespace psd
