/*
 * psd_oracle.c -- plain FP64 CPU oracle for the preconditioned steepest
 * descent (PSD) method of Feng, Salgado, Wang & Wise (arXiv:1607.01475).
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the slow, obviously-correct
 * reference against which the GPU library is checked.  It is loaded only by
 * the test-suite, by the smoke check and by the benchmark's CPU-baseline leg;
 * the product library never links, loads or calls it.  It shares no code,
 * header or table with the GPU path.
 *
 * Conventions
 *   - Periodic square/cubic box of side L, n cells per axis, h = L/n
 *     (Sec. 5.1).  Grid functions are stored as n^dim doubles, x fastest:
 *     idx = i + n*(j + n*k).  0-based cell i has centre (i+1/2)h, which is the
 *     paper's x_i = (i-1/2)h with 1-based i.
 *   - Half-integer positions: a value "at i+1/2" along an axis is stored at
 *     integer index i of that axis.  So a vertex (i+1/2, j+1/2[, k+1/2]) is
 *     stored at idx(i, j[, k]).
 *   - Every operator below is built from the four one-axis primitives of
 *     Sec. 5.1: the forward average A and difference D (integer -> half
 *     position), and the backward average a and difference d (half ->
 *     integer position).
 *   - Three dimensions: the paper only remarks that the operators extend
 *     (Remark after the discrete Sobolev lemma).  Reading used here: the
 *     collocated vertex derivative along axis a is D_a composed with the
 *     forward averages along both other axes, and the vertex-to-centre
 *     divergence uses d_a with the backward averages along the other axes.
 *     With this reading summation by parts holds exactly as in 2D.
 *   - No blocking, fusion or reordering beyond the definitions.
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>

typedef struct {
    int dim;      /* 2 or 3 */
    int n;        /* cells per axis */
    double L;     /* box side */
    int order;    /* 4: fourth-order equation, 6: sixth-order (u,w) system */
    double p;     /* p-Laplacian exponent, p >= 2 */
    double s;     /* s > 0 */
    double eps;   /* 0 < eps <= 1 */
    double lam;   /* lambda >= 0 (order 6 only) */
} orc_prob;

/* ------------------------------------------------------------------------ */
/* grid helpers                                                               */
/* ------------------------------------------------------------------------ */

static size_t ncell(const orc_prob *P) {
    size_t n = (size_t)P->n;
    return P->dim == 2 ? n * n : n * n * n;
}
static double hstep(const orc_prob *P) { return P->L / (double)P->n; }
static double hvol(const orc_prob *P) {
    double h = hstep(P);
    return P->dim == 2 ? h * h : h * h * h;
}
static int wrapi(int i, int n) { i %= n; return i < 0 ? i + n : i; }

/* index of the neighbour of cell `c` shifted by `off` along `axis` */
static size_t shifted(const orc_prob *P, size_t c, int axis, int off) {
    int n = P->n;
    int i = (int)(c % (size_t)n);
    int j = (int)((c / (size_t)n) % (size_t)n);
    int k = P->dim == 3 ? (int)(c / ((size_t)n * n)) : 0;
    if (axis == 0) i = wrapi(i + off, n);
    if (axis == 1) j = wrapi(j + off, n);
    if (axis == 2) k = wrapi(k + off, n);
    return (size_t)i + (size_t)n * ((size_t)j + (size_t)n * (size_t)k);
}

/* ------------------------------------------------------------------------ */
/* one-axis primitives (Sec. 5.1, averages and differences)                   */
/* ------------------------------------------------------------------------ */

/* forward average  A: out[i+1/2] = (v[i+1] + v[i]) / 2 */
static void op_A(const orc_prob *P, int axis, const double *v, double *out) {
    size_t N = ncell(P);
    for (size_t c = 0; c < N; ++c) out[c] = 0.5 * (v[shifted(P, c, axis, 1)] + v[c]);
}
/* forward difference D: out[i+1/2] = (v[i+1] - v[i]) / h */
static void op_D(const orc_prob *P, int axis, const double *v, double *out) {
    size_t N = ncell(P);
    double h = hstep(P);
    for (size_t c = 0; c < N; ++c) out[c] = (v[shifted(P, c, axis, 1)] - v[c]) / h;
}
/* backward average a: out[i] = (v[i+1/2] + v[i-1/2]) / 2 */
static void op_a(const orc_prob *P, int axis, const double *v, double *out) {
    size_t N = ncell(P);
    for (size_t c = 0; c < N; ++c) out[c] = 0.5 * (v[c] + v[shifted(P, c, axis, -1)]);
}
/* backward difference d: out[i] = (v[i+1/2] - v[i-1/2]) / h */
static void op_d(const orc_prob *P, int axis, const double *v, double *out) {
    size_t N = ncell(P);
    double h = hstep(P);
    for (size_t c = 0; c < N; ++c) out[c] = (v[c] - v[shifted(P, c, axis, -1)]) / h;
}

/* ------------------------------------------------------------------------ */
/* composite operators                                                       */
/* ------------------------------------------------------------------------ */

/* Collocated centre-to-vertex derivative along `axis` (Sec. 5.1, frak-D):
 * 2D: D_x A_y (and D_y A_x); 3D: D_a after the forward averages along the
 * two other axes. */
void orc_vgrad_axis(const orc_prob *P, int axis, const double *v, double *out) {
    size_t N = ncell(P);
    double *t1 = malloc(N * sizeof(double)), *t2 = malloc(N * sizeof(double));
    memcpy(t1, v, N * sizeof(double));
    for (int b = 0; b < P->dim; ++b) {
        if (b == axis) continue;
        op_A(P, b, t1, t2);
        memcpy(t1, t2, N * sizeof(double));
    }
    op_D(P, axis, t1, out);
    free(t1); free(t2);
}

/* Vertex-to-centre derivative along `axis` (Sec. 5.1, frak-d): d_a after the
 * backward averages along the other axes. */
void orc_vdiv_axis(const orc_prob *P, int axis, const double *v, double *out) {
    size_t N = ncell(P);
    double *t1 = malloc(N * sizeof(double)), *t2 = malloc(N * sizeof(double));
    memcpy(t1, v, N * sizeof(double));
    for (int b = 0; b < P->dim; ++b) {
        if (b == axis) continue;
        op_a(P, b, t1, t2);
        memcpy(t1, t2, N * sizeof(double));
    }
    op_d(P, axis, t1, out);
    free(t1); free(t2);
}

/* Standard Laplacian Delta_h = sum_a d_a D_a (Sec. 5.1). */
void orc_lap(const orc_prob *P, const double *v, double *out) {
    size_t N = ncell(P);
    double *t1 = malloc(N * sizeof(double)), *t2 = malloc(N * sizeof(double));
    memset(out, 0, N * sizeof(double));
    for (int a = 0; a < P->dim; ++a) {
        op_D(P, a, v, t1);
        op_d(P, a, t1, t2);
        for (size_t c = 0; c < N; ++c) out[c] += t2[c];
    }
    free(t1); free(t2);
}

/* Vertex gradient nabla_h^v v: G holds dim arrays of N values (Sec. 5.1). */
void orc_vgrad(const orc_prob *P, const double *v, double *G) {
    size_t N = ncell(P);
    for (int a = 0; a < P->dim; ++a) orc_vgrad_axis(P, a, v, G + (size_t)a * N);
}

/* Vertex-to-centre divergence of a vertex vector field F (dim arrays). */
void orc_vdiv(const orc_prob *P, const double *F, double *out) {
    size_t N = ncell(P);
    double *t = malloc(N * sizeof(double));
    memset(out, 0, N * sizeof(double));
    for (int a = 0; a < P->dim; ++a) {
        orc_vdiv_axis(P, a, F + (size_t)a * N, t);
        for (size_t c = 0; c < N; ++c) out[c] += t[c];
    }
    free(t);
}

/* |g|^{p-2} with the convention 0^0 = 1 (p = 2 gives the skew Laplacian). */
static double rpow(double g2, double p) {
    if (p == 2.0) return 1.0;
    if (g2 == 0.0) return 0.0;
    return pow(g2, 0.5 * (p - 2.0));
}

/* Discrete p-Laplacian  frak-d . ( |nabla_h^v v|^{p-2} nabla_h^v v )
 * (Sec. 5.1, discrete p-Laplacian operator). */
void orc_plap(const orc_prob *P, const double *v, double *out) {
    size_t N = ncell(P);
    int D = P->dim;
    double *G = malloc((size_t)D * N * sizeof(double));
    orc_vgrad(P, v, G);
    for (size_t c = 0; c < N; ++c) {
        double g2 = 0.0;
        for (int a = 0; a < D; ++a) g2 += G[a * N + c] * G[a * N + c];
        double r = rpow(g2, P->p);
        for (int a = 0; a < D; ++a) G[a * N + c] *= r;
    }
    orc_vdiv(P, G, out);
    free(G);
}

/* Linearised flux divergence used by the Hessian (second variation of the
 * discrete energy, Sec. 5.3):
 *   frak-d . ( |a|^{p-2} nabla xi + (p-2) |a|^{p-4} (a . nabla xi) a ),
 * a = nabla_h^v u.  The (p-2)|a|^{p-4} term is taken as 0 where a = 0. */
void orc_plap_lin(const orc_prob *P, const double *u, const double *xi, double *out) {
    size_t N = ncell(P);
    int D = P->dim;
    double *A = malloc((size_t)D * N * sizeof(double));
    double *B = malloc((size_t)D * N * sizeof(double));
    orc_vgrad(P, u, A);
    orc_vgrad(P, xi, B);
    for (size_t c = 0; c < N; ++c) {
        double a2 = 0.0, ab = 0.0;
        for (int a = 0; a < D; ++a) {
            a2 += A[a * N + c] * A[a * N + c];
            ab += A[a * N + c] * B[a * N + c];
        }
        double r = rpow(a2, P->p);
        double r4 = (a2 == 0.0 || P->p == 2.0) ? 0.0 : (P->p - 2.0) * pow(a2, 0.5 * (P->p - 4.0));
        for (int a = 0; a < D; ++a) B[a * N + c] = r * B[a * N + c] + r4 * ab * A[a * N + c];
    }
    orc_vdiv(P, B, out);
    free(A); free(B);
}

/* ------------------------------------------------------------------------ */
/* Fourier transforms: brute-force DFT and a plain mixed-radix FFT            */
/* sign = -1: forward  X_k = sum_j x_j e^{-2 pi i jk/n}; sign = +1: inverse   */
/* without 1/n.  Used only to apply constant-coefficient operators (Sec. 6). */
/* ------------------------------------------------------------------------ */

void orc_dft1(int n, const double *xr, const double *xi, double *yr, double *yi, int sign) {
    for (int k = 0; k < n; ++k) {
        long double sr = 0.0L, si = 0.0L;
        for (int j = 0; j < n; ++j) {
            long m = ((long)j * k) % n;
            long double ang = (long double)sign * 2.0L * 3.14159265358979323846264338327950288L
                              * (long double)m / (long double)n;
            long double c = cosl(ang), s = sinl(ang);
            sr += xr[j] * c - xi[j] * s;
            si += xr[j] * s + xi[j] * c;
        }
        yr[k] = (double)sr;
        yi[k] = (double)si;
    }
}

/* Recursive decimation in time by the smallest prime factor r of n (a
 * plain DFT when n is prime).  tw[t] = e^{sign 2 pi i t / ntop} is the root
 * table of the top-level length; a sub-transform of length n uses the
 * stride ntop/n into it.  ws is scratch of at least 4n doubles. */
static void fft_rec(int n, double *xr, double *xi, const double *twr, const double *twi,
                    int ntop, double *ws) {
    if (n == 1) return;
    int r = 0;
    for (int f = 2; f * f <= n; ++f) if (n % f == 0) { r = f; break; }
    int tstride = ntop / n;
    if (r == 0) { /* prime length: plain DFT with the table */
        double *yr = ws, *yi = ws + n;
        for (int k = 0; k < n; ++k) {
            double sr = 0.0, si = 0.0;
            for (int j = 0; j < n; ++j) {
                int m = (int)(((long)j * k) % n) * tstride;
                sr += xr[j] * twr[m] - xi[j] * twi[m];
                si += xr[j] * twi[m] + xi[j] * twr[m];
            }
            yr[k] = sr; yi[k] = si;
        }
        memcpy(xr, yr, n * sizeof(double)); memcpy(xi, yi, n * sizeof(double));
        return;
    }
    int m = n / r;
    double *sr = ws, *si = ws + n, *child = ws + 2 * n;
    /* split into r decimated sub-sequences x[q + r*j], transform each */
    for (int q = 0; q < r; ++q)
        for (int j = 0; j < m; ++j) { sr[q * m + j] = xr[q + r * j]; si[q * m + j] = xi[q + r * j]; }
    for (int q = 0; q < r; ++q) fft_rec(m, sr + q * m, si + q * m, twr, twi, ntop, child);
    /* combine: X[k] = sum_q e^{sign 2 pi i q k / n} S_q[k mod m] */
    for (int k = 0; k < n; ++k) {
        double ar = 0.0, ai = 0.0;
        for (int q = 0; q < r; ++q) {
            int t = (int)(((long)q * k) % n) * tstride;
            double br = sr[q * m + (k % m)], bi = si[q * m + (k % m)];
            ar += br * twr[t] - bi * twi[t];
            ai += br * twi[t] + bi * twr[t];
        }
        xr[k] = ar; xi[k] = ai;
    }
}

typedef struct { int n; double *twr, *twi, *ws; } fft_plan1;

static fft_plan1 plan1_make(int n, int sign) {
    fft_plan1 pl;
    pl.n = n;
    pl.twr = malloc(n * sizeof(double));
    pl.twi = malloc(n * sizeof(double));
    pl.ws = malloc((size_t)(6 * n + 8) * sizeof(double));
    for (int t = 0; t < n; ++t) {
        long double ang = (long double)sign * 2.0L * 3.14159265358979323846264338327950288L
                          * (long double)t / (long double)n;
        pl.twr[t] = (double)cosl(ang);
        pl.twi[t] = (double)sinl(ang);
    }
    return pl;
}
static void plan1_free(fft_plan1 *pl) { free(pl->twr); free(pl->twi); free(pl->ws); }

void orc_fft1(int n, double *xr, double *xi, int sign) {
    fft_plan1 pl = plan1_make(n, sign);
    fft_rec(n, xr, xi, pl.twr, pl.twi, n, pl.ws);
    plan1_free(&pl);
}

/* multi-dimensional transform, one axis after the other (in place) */
void orc_fftn(int dim, int n, double *re, double *im, int sign, int naive) {
    size_t N = (size_t)n * n * (dim == 3 ? (size_t)n : 1);
    double *lr = malloc(n * sizeof(double)), *li = malloc(n * sizeof(double));
    double *yr = malloc(n * sizeof(double)), *yi = malloc(n * sizeof(double));
    fft_plan1 pl = plan1_make(n, sign);
    for (int axis = 0; axis < dim; ++axis) {
        size_t stride = axis == 0 ? 1 : (axis == 1 ? (size_t)n : (size_t)n * n);
        for (size_t base = 0; base < N; ++base) {
            /* base must have coordinate 0 along `axis` */
            if ((base / stride) % (size_t)n != 0) continue;
            for (int t = 0; t < n; ++t) { lr[t] = re[base + t * stride]; li[t] = im[base + t * stride]; }
            if (naive) {
                orc_dft1(n, lr, li, yr, yi, sign);
                memcpy(lr, yr, n * sizeof(double)); memcpy(li, yi, n * sizeof(double));
            } else {
                fft_rec(n, lr, li, pl.twr, pl.twi, n, pl.ws);
            }
            for (int t = 0; t < n; ++t) { re[base + t * stride] = lr[t]; im[base + t * stride] = li[t]; }
        }
    }
    plan1_free(&pl);
    free(lr); free(li); free(yr); free(yi);
}

/* ------------------------------------------------------------------------ */
/* constant-coefficient operators and their Fourier symbols                   */
/* ------------------------------------------------------------------------ */

/* Eigenvalues of a periodic, translation-invariant linear operator are the
 * DFT of its response to a unit impulse at cell 0.  The symbols of -Delta_h
 * and of the preconditioners are taken this way from the operator
 * definitions themselves (no separate closed-form formula in this file). */
static void impulse_symbol_lap(const orc_prob *P, double *kappa) {
    size_t N = ncell(P);
    double *e = calloc(N, sizeof(double)), *im = calloc(N, sizeof(double));
    double *le = malloc(N * sizeof(double));
    e[0] = 1.0;
    orc_lap(P, e, le);
    for (size_t c = 0; c < N; ++c) le[c] = -le[c];
    orc_fftn(P->dim, P->n, le, im, -1, 0);
    /* symmetric stencil: the symbol is real */
    memcpy(kappa, le, N * sizeof(double));
    free(e); free(im); free(le);
}

/* Symbol of -Delta_h (exposed for tests). */
void orc_symbol_neglap(const orc_prob *P, double *kappa) { impulse_symbol_lap(P, kappa); }

/* Symbol of the preconditioner L_h:
 *   order 4 (Sec. 5.3):  1 + s*kappa + s*eps^2*kappa^2
 *   order 6 (Sec. 5.4):  s*lam + s*kappa + s*eps^2*kappa^2 + 1/kappa  (k != 0)
 * with kappa the symbol of -Delta_h, so that L_h = I - s Delta_h + s eps^2 Delta_h^2
 * (+ T_h for order 6).  The k = 0 entry of order 6 is set to +inf (the
 * operator acts on mean-zero functions). */
void orc_symbol_precond(const orc_prob *P, double *sigma) {
    size_t N = ncell(P);
    impulse_symbol_lap(P, sigma);
    double s = P->s, e2 = P->eps * P->eps;
    for (size_t c = 0; c < N; ++c) {
        double k = sigma[c];
        if (P->order == 4) sigma[c] = 1.0 + s * k + s * e2 * k * k;
        else sigma[c] = (c == 0) ? INFINITY : s * P->lam + s * k + s * e2 * k * k + 1.0 / k;
    }
}

/* Apply the inverse of a diagonal-in-Fourier operator with symbol `sym`
 * to a real field:  out = IDFT( DFT(in) / sym ).  Entries with sym = inf
 * are mapped to zero. */
static void fourier_divide(const orc_prob *P, const double *sym, const double *in, double *out) {
    size_t N = ncell(P);
    double *re = malloc(N * sizeof(double)), *im = calloc(N, sizeof(double));
    memcpy(re, in, N * sizeof(double));
    orc_fftn(P->dim, P->n, re, im, -1, 0);
    for (size_t c = 0; c < N; ++c) {
        if (isinf(sym[c])) { re[c] = 0.0; im[c] = 0.0; }
        else { re[c] /= sym[c]; im[c] /= sym[c]; }
    }
    orc_fftn(P->dim, P->n, re, im, +1, 0);
    for (size_t c = 0; c < N; ++c) out[c] = re[c] / (double)N;
    free(re); free(im);
}

/* Search direction: solve L_h d = r (Sec. 6.1 and Sec. 6.2). */
void orc_precond(const orc_prob *P, const double *r, double *d) {
    size_t N = ncell(P);
    double *sig = malloc(N * sizeof(double));
    orc_symbol_precond(P, sig);
    fourier_divide(P, sig, r, d);
    free(sig);
}

/* T_h = -Delta_h^{-1} on mean-zero functions (Sec. 5.1); the mean of the
 * input is discarded (k = 0 mode set to zero). */
void orc_T(const orc_prob *P, const double *z, double *out) {
    size_t N = ncell(P);
    double *kap = malloc(N * sizeof(double));
    impulse_symbol_lap(P, kap);
    kap[0] = INFINITY;
    fourier_divide(P, kap, z, out);
    free(kap);
}

/* ------------------------------------------------------------------------ */
/* inner products and norms (Sec. 5.1)                                        */
/* ------------------------------------------------------------------------ */

double orc_ip(const orc_prob *P, const double *a, const double *b) {
    size_t N = ncell(P);
    double s = 0.0;
    for (size_t c = 0; c < N; ++c) s += a[c] * b[c];
    return hvol(P) * s;
}
static double mean_of(const orc_prob *P, const double *a) {
    size_t N = ncell(P);
    double s = 0.0;
    for (size_t c = 0; c < N; ++c) s += a[c];
    return s / (double)N;
}
double orc_maxabs(const orc_prob *P, const double *a) {
    size_t N = ncell(P);
    double m = 0.0;
    for (size_t c = 0; c < N; ++c) if (fabs(a[c]) > m) m = fabs(a[c]);
    return m;
}

/* ------------------------------------------------------------------------ */
/* fourth-order problem                                                       */
/* ------------------------------------------------------------------------ */

/* N_h[u] = u - s frak-d.(|nabla u|^{p-2} nabla u) + s eps^2 Delta_h^2 u
 * (Sec. 5.3, discrete fourth-order equation). */
void orc_N4(const orc_prob *P, const double *u, double *out) {
    size_t N = ncell(P);
    double *pl = malloc(N * sizeof(double)), *l1 = malloc(N * sizeof(double)),
           *l2 = malloc(N * sizeof(double));
    orc_plap(P, u, pl);
    orc_lap(P, u, l1);
    orc_lap(P, l1, l2);
    double s = P->s, se2 = P->s * P->eps * P->eps;
    for (size_t c = 0; c < N; ++c) out[c] = u[c] - s * pl[c] + se2 * l2[c];
    free(pl); free(l1); free(l2);
}

/* Discrete energy (Sec. 5.3):
 *   E_h = 1/2 ||u-f||_2^2 + s/p ||nabla_h^v u||_p^p + s eps^2/2 ||Delta_h u||_2^2,
 * with the vertex sum <.,.> = h^dim sum over vertices (one vertex per cell). */
double orc_energy4(const orc_prob *P, const double *f, const double *u) {
    size_t N = ncell(P);
    int D = P->dim;
    double *G = malloc((size_t)D * N * sizeof(double)), *l1 = malloc(N * sizeof(double));
    orc_vgrad(P, u, G);
    orc_lap(P, u, l1);
    double e1 = 0.0, e2 = 0.0, e3 = 0.0;
    for (size_t c = 0; c < N; ++c) {
        double g2 = 0.0;
        for (int a = 0; a < D; ++a) g2 += G[a * N + c] * G[a * N + c];
        e1 += (u[c] - f[c]) * (u[c] - f[c]);
        e2 += pow(g2, 0.5 * P->p);
        e3 += l1[c] * l1[c];
    }
    free(G); free(l1);
    return hvol(P) * (0.5 * e1 + P->s / P->p * e2 + 0.5 * P->s * P->eps * P->eps * e3);
}

/* Residual r = f - N_h[u] = -delta E_h[u] (Sec. 5.3 and Sec. 6.1). */
void orc_residual4(const orc_prob *P, const double *f, const double *u, double *r) {
    size_t N = ncell(P);
    orc_N4(P, u, r);
    for (size_t c = 0; c < N; ++c) r[c] = f[c] - r[c];
}

/* ------------------------------------------------------------------------ */
/* sixth-order problem (Sec. 4 and Sec. 5.4; SPFC form Sec. 6.2)              */
/* ------------------------------------------------------------------------ */

/* Nonlinear part shared by both forms: s lam u - s plap(u) + s eps^2 Delta_h^2 u */
static void stencil6(const orc_prob *P, const double *u, double *out) {
    size_t N = ncell(P);
    double *pl = malloc(N * sizeof(double)), *l1 = malloc(N * sizeof(double)),
           *l2 = malloc(N * sizeof(double));
    orc_plap(P, u, pl);
    orc_lap(P, u, l1);
    orc_lap(P, l1, l2);
    double s = P->s, se2 = P->s * P->eps * P->eps;
    for (size_t c = 0; c < N; ++c) out[c] = s * P->lam * u[c] - s * pl[c] + se2 * l2[c];
    free(pl); free(l1); free(l2);
}

/* Reduced residual of the sixth-order problem on the mean-zero space:
 *   rho = P0[ f - s lam u + s plap(u) - s eps^2 Delta_h^2 u - T_h(u - g) ],
 * i.e. minus the gradient of the mean-zero energy at nu = u - mean(g)
 * (Sec. 4: first variation; Sec. 6.2: N_h with T_h[-nu + g]). */
void orc_residual6(const orc_prob *P, const double *f, const double *g, const double *u,
                   double *rho) {
    size_t N = ncell(P);
    double *st = malloc(N * sizeof(double)), *z = malloc(N * sizeof(double)),
           *tz = malloc(N * sizeof(double));
    stencil6(P, u, st);
    for (size_t c = 0; c < N; ++c) z[c] = u[c] - g[c];
    orc_T(P, z, tz);
    for (size_t c = 0; c < N; ++c) rho[c] = f[c] - st[c] - tz[c];
    double m = mean_of(P, rho);
    for (size_t c = 0; c < N; ++c) rho[c] -= m;
    free(st); free(z); free(tz);
}

/* Sixth-order discrete energy (Sec. 5.4) evaluated at nu = u - mean(g):
 *   1/2 ||nu-g+gbar||_{-1}^2 + lam s/2 ||nu+gbar||^2 - (nu,f) + s/p ||grad nu||_p^p
 *   + s eps^2/2 ||Delta_h nu||^2 */
double orc_energy6(const orc_prob *P, const double *f, const double *g, const double *u) {
    size_t N = ncell(P);
    int D = P->dim;
    double gbar = mean_of(P, g);
    double *z = malloc(N * sizeof(double)), *tz = malloc(N * sizeof(double));
    double *nu = malloc(N * sizeof(double));
    for (size_t c = 0; c < N; ++c) { nu[c] = u[c] - gbar; z[c] = nu[c] - g[c] + gbar; }
    orc_T(P, z, tz);
    double *G = malloc((size_t)D * N * sizeof(double)), *l1 = malloc(N * sizeof(double));
    orc_vgrad(P, nu, G);
    orc_lap(P, nu, l1);
    double eneg = 0.0, el2 = 0.0, ef = 0.0, ep = 0.0, el = 0.0;
    for (size_t c = 0; c < N; ++c) {
        double g2 = 0.0;
        for (int a = 0; a < D; ++a) g2 += G[a * N + c] * G[a * N + c];
        eneg += z[c] * tz[c];
        el2 += (nu[c] + gbar) * (nu[c] + gbar);
        ef += nu[c] * f[c];
        ep += pow(g2, 0.5 * P->p);
        el += l1[c] * l1[c];
    }
    free(z); free(tz); free(nu); free(G); free(l1);
    return hvol(P) * (0.5 * eneg + 0.5 * P->lam * P->s * el2 - ef + P->s / P->p * ep
                      + 0.5 * P->s * P->eps * P->eps * el);
}

/* Chemical potential after convergence (Sec. 4): w = T_h[g - u] + s lam gbar - fbar. */
void orc_w_from_u(const orc_prob *P, const double *f, const double *g, const double *u,
                  double *w) {
    size_t N = ncell(P);
    double *z = malloc(N * sizeof(double));
    for (size_t c = 0; c < N; ++c) z[c] = g[c] - u[c];
    orc_T(P, z, w);
    double shift = P->s * P->lam * mean_of(P, g) - mean_of(P, f);
    for (size_t c = 0; c < N; ++c) w[c] += shift;
    free(z);
}

/* Residuals of the mixed system (Sec. 5.4):
 *   r1 = g - u + Delta_h w,  r2 = f - (s lam u - s plap u + s eps^2 Delta_h^2 u - w). */
void orc_mixed_residuals(const orc_prob *P, const double *f, const double *g, const double *u,
                         const double *w, double *r1, double *r2) {
    size_t N = ncell(P);
    double *lw = malloc(N * sizeof(double)), *st = malloc(N * sizeof(double));
    orc_lap(P, w, lw);
    stencil6(P, u, st);
    for (size_t c = 0; c < N; ++c) {
        r1[c] = g[c] - u[c] + lw[c];
        r2[c] = f[c] - (st[c] - w[c]);
    }
    free(lw); free(st);
}

/* ------------------------------------------------------------------------ */
/* line search (Sec. 6.1: q(alpha) = (N_h[u + alpha d] - f, d)_2)             */
/* ------------------------------------------------------------------------ */

/* Coefficients of the cubic q for p = 4 (h^dim factor dropped throughout).
 * With a = nabla u, b = nabla d at vertices:
 *   c0 = q(0) = -(r, d)               (r the current residual; the exact
 *                                      value of q(0), no cancellation)
 *   c1 = (d,d)* + s sum_V (|a|^2|b|^2 + 2 (a.b)^2) + s eps^2 (Delta d, Delta d)
 *   c2 = 3 s sum_V (a.b)|b|^2
 *   c3 = s sum_V |b|^4
 * (*) order 4: (d,d); order 6: s lam (d,d) + (T_h d, d).
 * These follow from expanding |a + alpha b|^2 (a + alpha b).b and summation
 * by parts, which turns (-frak-d.F, d)_2 into <F, nabla d>. */
void orc_ls_coeffs4(const orc_prob *P, const double *u, const double *d, const double *r,
                    double *c) {
    size_t N = ncell(P);
    int D = P->dim;
    double *A = malloc((size_t)D * N * sizeof(double)), *B = malloc((size_t)D * N * sizeof(double));
    double *ld = malloc(N * sizeof(double));
    orc_vgrad(P, u, A);
    orc_vgrad(P, d, B);
    orc_lap(P, d, ld);
    double rd = 0.0, dd = 0.0, S2 = 0.0, S3 = 0.0, S4 = 0.0, S5 = 0.0, P4 = 0.0;
    for (size_t c2 = 0; c2 < N; ++c2) {
        double a2 = 0.0, b2 = 0.0, ab = 0.0;
        for (int a = 0; a < D; ++a) {
            a2 += A[a * N + c2] * A[a * N + c2];
            b2 += B[a * N + c2] * B[a * N + c2];
            ab += A[a * N + c2] * B[a * N + c2];
        }
        rd += r[c2] * d[c2];
        dd += d[c2] * d[c2];
        S2 += a2 * b2; S3 += ab * ab; S4 += ab * b2; S5 += b2 * b2;
        P4 += ld[c2] * ld[c2];
    }
    double s = P->s, se2 = P->s * P->eps * P->eps;
    double lin = dd;
    if (P->order == 6) {
        double *td = malloc(N * sizeof(double));
        orc_T(P, d, td);
        double tdd = 0.0;
        for (size_t c2 = 0; c2 < N; ++c2) tdd += td[c2] * d[c2];
        lin = s * P->lam * dd + tdd;
        free(td);
    }
    c[0] = -rd;
    c[1] = lin + s * (S2 + 2.0 * S3) + se2 * P4;
    c[2] = 3.0 * s * S4;
    c[3] = s * S5;
    free(A); free(B); free(ld);
}

/* General p: q(alpha) and q'(alpha) evaluated from the definition
 *   q(alpha)  = (N_h[u + alpha d] - f, d)_2            (order 4)
 *   q'(alpha) = second variation at u + alpha d in direction (d, d)
 * (h^dim factor dropped).  Order 6 uses its N_h with the T_h term. */
void orc_q_eval(const orc_prob *P, const double *f, const double *g, const double *u,
                const double *d, double alpha, double *q, double *dq) {
    size_t N = ncell(P);
    double *v = malloc(N * sizeof(double)), *r = malloc(N * sizeof(double));
    for (size_t c = 0; c < N; ++c) v[c] = u[c] + alpha * d[c];
    if (P->order == 4) orc_residual4(P, f, v, r);
    else orc_residual6(P, f, g, v, r);
    double sq = 0.0;
    for (size_t c = 0; c < N; ++c) sq -= r[c] * d[c];
    /* second variation (Sec. 5.3): (d,d) + s<|a|^{p-2} b, b> + (p-2)s<|a|^{p-4}(a.b)^2>
     * + s eps^2 (Delta d, Delta d); evaluated as (-s plap_lin(v; d) + ..., d). */
    double *pl = malloc(N * sizeof(double)), *l1 = malloc(N * sizeof(double)),
           *l2 = malloc(N * sizeof(double));
    orc_plap_lin(P, v, d, pl);
    orc_lap(P, d, l1);
    orc_lap(P, l1, l2);
    double s = P->s, se2 = P->s * P->eps * P->eps, sdq = 0.0;
    for (size_t c = 0; c < N; ++c) sdq += (-s * pl[c] + se2 * l2[c]) * d[c];
    double dd = 0.0;
    for (size_t c = 0; c < N; ++c) dd += d[c] * d[c];
    if (P->order == 4) sdq += dd;
    else {
        double *td = malloc(N * sizeof(double));
        orc_T(P, d, td);
        double tdd = 0.0;
        for (size_t c = 0; c < N; ++c) tdd += td[c] * d[c];
        sdq += s * P->lam * dd + tdd;
        free(td);
    }
    *q = sq; *dq = sdq;
    free(v); free(r); free(pl); free(l1); free(l2);
}

/* Root of the strictly increasing q (Sec. 6.1: unique root).  The paper
 * does not fix the method; rule used on both sides of the test:
 *   x = -q(0)/q'(0); double x until q(x) > 0 (bracket [lo, hi]);
 *   Newton from hi, replaced by bisection whenever it leaves (lo, hi);
 *   stop when |q| <= 1e-16 (|q(0)| + q'(0) x) or |dx| <= 1e-15 x (<= 100 steps). */
typedef void (*qfun)(void *ctx, double x, double *q, double *dq);

static double root_rule(qfun fn, void *ctx, double c0, double c1, int *evals) {
    double lo = 0.0, hi = INFINITY, x = -c0 / c1, qx = 0.0, dqx = 0.0;
    int ev = 0;
    for (int it = 0; it < 200; ++it) {
        fn(ctx, x, &qx, &dqx); ++ev;
        if (qx > 0.0) { hi = x; break; }
        if (qx == 0.0) { if (evals) *evals = ev; return x; }
        lo = x;
        x *= 2.0;
    }
    for (int it = 0; it < 100; ++it) {
        if (fabs(qx) <= 1e-16 * (fabs(c0) + c1 * x)) break;
        double xn = x - qx / dqx;
        if (!(xn > lo && xn < hi)) xn = 0.5 * (lo + hi);
        if (fabs(xn - x) <= 1e-15 * x) { x = xn; break; }
        x = xn;
        fn(ctx, x, &qx, &dqx); ++ev;
        if (qx > 0.0) hi = x;
        else if (qx < 0.0) lo = x;
        else break;
    }
    if (evals) *evals = ev;
    return x;
}

static void cubic_fn(void *ctx, double x, double *q, double *dq) {
    const double *c = (const double *)ctx;
    *q = c[0] + x * (c[1] + x * (c[2] + x * c[3]));
    *dq = c[1] + x * (2.0 * c[2] + 3.0 * c[3] * x);
}

double orc_root_cubic(const double *c, int *evals) {
    return root_rule(cubic_fn, (void *)c, c[0], c[1], evals);
}

typedef struct {
    const orc_prob *P; const double *f, *g, *u, *d;
} qctx;

static void grid_fn(void *ctx, double x, double *q, double *dq) {
    qctx *C = (qctx *)ctx;
    orc_q_eval(C->P, C->f, C->g, C->u, C->d, x, q, dq);
}

/* ------------------------------------------------------------------------ */
/* the PSD loop (Sec. 2.2 search direction, update and exact line search;    */
/* loop shape of the linear algorithm in Sec. 2.1)                            */
/* ------------------------------------------------------------------------ */

/* Solve N_h[u] = f (order 4) or the mixed system (order 6) by PSD.
 *   u: in = u0, out = final iterate.  w (order 6, may be NULL): out.
 *   Stop when ||r||_inf <= tol (absolute, FP64) after an update, or after
 *   max_iter updates.  Order 6 uses the reduced residual rho.
 *   hist (may be NULL): 4 doubles per update: alpha, ||r||_inf, ||r||_2, E_h.
 *   out_stats (may be NULL): [0] final ||r||_inf, [1] final ||r||_2, [2] E_h.
 * Returns the number of updates, or -1 on a bad argument, -2 when the start
 * of an order-6 solve does not have mean(u0) = mean(g), -3 when q(0) >= 0
 * with a residual above tolerance (not a descent direction). */
int orc_solve(const orc_prob *P, const double *f, const double *g, double *u, double *w,
              double tol, int max_iter, double *hist, double *out_stats) {
    if (!P || !f || !u || P->n < 2 || (P->dim != 2 && P->dim != 3)) return -1;
    if (P->order == 6 && !g) return -1;
    size_t N = ncell(P);
    if (P->order == 6) {
        double gb = mean_of(P, g), ub = mean_of(P, u);
        if (fabs(ub - gb) > 1e-12 * (1.0 + fabs(gb))) return -2;
    }
    double *r = malloc(N * sizeof(double)), *d = malloc(N * sizeof(double));
    if (P->order == 4) orc_residual4(P, f, u, r); else orc_residual6(P, f, g, u, r);
    double rinf = orc_maxabs(P, r);
    int k = 0, status = 0;
    while (rinf > tol && k < max_iter) {
        orc_precond(P, r, d);
        double alpha;
        if (P->p == 4.0) {
            double c[4];
            orc_ls_coeffs4(P, u, d, r, c);
            if (!(c[0] < 0.0)) { status = -3; break; }
            alpha = orc_root_cubic(c, NULL);
        } else {
            qctx C = {P, f, g, u, d};
            double q0, dq0;
            orc_q_eval(P, f, g, u, d, 0.0, &q0, &dq0);
            /* q(0) exactly as in the cubic case */
            q0 = -orc_ip(P, r, d) / hvol(P);
            if (!(q0 < 0.0)) { status = -3; break; }
            alpha = root_rule(grid_fn, &C, q0, dq0, NULL);
        }
        for (size_t c = 0; c < N; ++c) u[c] += alpha * d[c];
        ++k;
        if (P->order == 4) orc_residual4(P, f, u, r); else orc_residual6(P, f, g, u, r);
        rinf = orc_maxabs(P, r);
        if (hist) {
            hist[4 * (k - 1) + 0] = alpha;
            hist[4 * (k - 1) + 1] = rinf;
            hist[4 * (k - 1) + 2] = sqrt(orc_ip(P, r, r));
            hist[4 * (k - 1) + 3] = P->order == 4 ? orc_energy4(P, f, u) : orc_energy6(P, f, g, u);
        }
    }
    if (out_stats) {
        out_stats[0] = rinf;
        out_stats[1] = sqrt(orc_ip(P, r, r));
        out_stats[2] = P->order == 4 ? orc_energy4(P, f, u) : orc_energy6(P, f, g, u);
    }
    if (P->order == 6 && w) orc_w_from_u(P, f, g, u, w);
    free(r); free(d);
    return status < 0 ? status : k;
}

/* ------------------------------------------------------------------------ */
/* adjoint of the converged fourth-order solve                               */
/* ------------------------------------------------------------------------ */

/* Hessian of the discrete energy at u as an operator (second variation,
 * Sec. 5.3):  H xi = xi - s frak-d.(|a|^{p-2} nabla xi + (p-2)|a|^{p-4}(a.nabla xi) a)
 *                    + s eps^2 Delta_h^2 xi,   a = nabla_h^v u,
 * so that delta^2 E_h[u](xi, eta) = (H xi, eta)_2. */
void orc_hessvec(const orc_prob *P, const double *u, const double *xi, double *out) {
    size_t N = ncell(P);
    double *pl = malloc(N * sizeof(double)), *l1 = malloc(N * sizeof(double)),
           *l2 = malloc(N * sizeof(double));
    orc_plap_lin(P, u, xi, pl);
    orc_lap(P, xi, l1);
    orc_lap(P, l1, l2);
    double s = P->s, se2 = P->s * P->eps * P->eps;
    for (size_t c = 0; c < N; ++c) out[c] = xi[c] - s * pl[c] + se2 * l2[c];
    free(pl); free(l1); free(l2);
}

/* Sensitivities of N_h with respect to its parameters at u:
 *   dN/ds   = -plap(u) + eps^2 Delta_h^2 u,   dN/deps = 2 s eps Delta_h^2 u. */
void orc_dN_dparams(const orc_prob *P, const double *u, double *dNds, double *dNdeps) {
    size_t N = ncell(P);
    double *pl = malloc(N * sizeof(double)), *l1 = malloc(N * sizeof(double)),
           *l2 = malloc(N * sizeof(double));
    orc_plap(P, u, pl);
    orc_lap(P, u, l1);
    orc_lap(P, l1, l2);
    for (size_t c = 0; c < N; ++c) {
        dNds[c] = -pl[c] + P->eps * P->eps * l2[c];
        dNdeps[c] = 2.0 * P->s * P->eps * l2[c];
    }
    free(pl); free(l1); free(l2);
}

/* Adjoint solve by preconditioned CG:  H lam = gu  (H symmetric positive
 * definite, preconditioned by L_h^{-1}).  gu is the plain partial derivative
 * of the loss with respect to the cell values of u*.  Outputs the plain
 * partial derivatives dJ/df = lam, dJ/ds = -lam.dN/ds, dJ/deps = -lam.dN/deps.
 * Stops at ||res||_2 <= rtol ||gu||_2.  Returns CG iterations (or -1). */
int orc_adjoint(const orc_prob *P, const double *u, const double *gu, double rtol, int max_iter,
                double *lam, double *dJds, double *dJdeps) {
    if (P->order != 4) return -1;
    size_t N = ncell(P);
    double *res = malloc(N * sizeof(double)), *z = malloc(N * sizeof(double)),
           *pv = malloc(N * sizeof(double)), *Hp = malloc(N * sizeof(double));
    memset(lam, 0, N * sizeof(double));
    memcpy(res, gu, N * sizeof(double));
    double g0 = 0.0;
    for (size_t c = 0; c < N; ++c) g0 += gu[c] * gu[c];
    g0 = sqrt(g0);
    orc_precond(P, res, z);
    memcpy(pv, z, N * sizeof(double));
    double rz = 0.0;
    for (size_t c = 0; c < N; ++c) rz += res[c] * z[c];
    int it = 0;
    for (; it < max_iter; ++it) {
        double rn = 0.0;
        for (size_t c = 0; c < N; ++c) rn += res[c] * res[c];
        if (sqrt(rn) <= rtol * g0) break;
        orc_hessvec(P, u, pv, Hp);
        double pHp = 0.0;
        for (size_t c = 0; c < N; ++c) pHp += pv[c] * Hp[c];
        double a = rz / pHp;
        for (size_t c = 0; c < N; ++c) { lam[c] += a * pv[c]; res[c] -= a * Hp[c]; }
        orc_precond(P, res, z);
        double rz2 = 0.0;
        for (size_t c = 0; c < N; ++c) rz2 += res[c] * z[c];
        double b = rz2 / rz;
        rz = rz2;
        for (size_t c = 0; c < N; ++c) pv[c] = z[c] + b * pv[c];
    }
    double *ds = malloc(N * sizeof(double)), *de = malloc(N * sizeof(double));
    orc_dN_dparams(P, u, ds, de);
    double js = 0.0, je = 0.0;
    for (size_t c = 0; c < N; ++c) { js -= lam[c] * ds[c]; je -= lam[c] * de[c]; }
    *dJds = js; *dJdeps = je;
    free(res); free(z); free(pv); free(Hp); free(ds); free(de);
    return it;
}

/* Dense Cholesky solve A x = b (A symmetric positive definite, m x m,
 * row-major, overwritten).  Returns 0 on success, -1 if not SPD. */
int orc_cholesky_solve(int m, double *A, double *b) {
    for (int j = 0; j < m; ++j) {
        double dsum = A[j * m + j];
        for (int k = 0; k < j; ++k) dsum -= A[j * m + k] * A[j * m + k];
        if (!(dsum > 0.0)) return -1;
        double Ljj = sqrt(dsum);
        A[j * m + j] = Ljj;
        for (int i = j + 1; i < m; ++i) {
            double v = A[i * m + j];
            for (int k = 0; k < j; ++k) v -= A[i * m + k] * A[j * m + k];
            A[i * m + j] = v / Ljj;
        }
    }
    for (int i = 0; i < m; ++i) {           /* L y = b */
        double v = b[i];
        for (int k = 0; k < i; ++k) v -= A[i * m + k] * b[k];
        b[i] = v / A[i * m + i];
    }
    for (int i = m - 1; i >= 0; --i) {      /* L^T x = y */
        double v = b[i];
        for (int k = i + 1; k < m; ++k) v -= A[k * m + i] * b[k];
        b[i] = v / A[i * m + i];
    }
    return 0;
}
