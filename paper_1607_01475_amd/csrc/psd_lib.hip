// psd_lib.hip -- host runtime and C ABI of the gfx950 PSD solver.
//
// One handle holds a batch of instances (same dim, order and p; sizes and
// coefficients may differ).  At creation it builds, per instance, the
// symbol table S[k] = (4/h^2) sin^2(pi k/n) of -Delta_h along one axis
// (appendix: eigenvalues of the difference operators), FP32 and FP64
// twiddle tables, all work buffers, and the task tables of every pass.
// One PSD iteration (Sec. 2.2 / Sec. 6) is the launch sequence
//   rows R2C -> [cols fwd (3D)] -> cols fwd + 1/sigma + inv -> [cols inv]
//   -> rows C2R   (search direction d, Sec. 6.1 / 6.2)
//   -> line-search sums -> line-search finalize (alpha, Sec. 6.1)
//   -> update + residual -> residual finalize (stop test)
// all enqueued on one stream; in graph mode a chunk of iterations is
// captured once into a HIP graph and replayed until the device flag is set.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "psd_kernels.hpp"
#include "../../include/psd.h"

using namespace psd;

namespace {

thread_local std::string g_create_error;

// launch group of one transform length inside a pass
struct NPart {
  int n = 0, off = 0, cnt = 0;
  size_t lds = 0;
};

struct Range {
  int off = 0, cnt = 0;
  size_t lds = 0;
  std::vector<NPart> parts;   // FFT passes: tasks grouped by n, one launch per group
};

struct FftTasks {  // task ranges of one spectral application
  Range r2c, coly_f, colz, coly_i, c2r;
};

size_t ceil_div(size_t a, size_t b) { return (a + b - 1) / b; }

bool n_supported(int n) {
  switch (n) {
    case 16: case 32: case 48: case 64: case 96: case 128: case 192: case 256: case 384: case 512:
    case 1024:
      return true;
    default:
      return false;
  }
}

template <typename T>
int host_row_lines(int n, int sel) {
  switch (n) {
#define C(NN) \
  case NN: return sel == 0 ? row_lines<T, NN, 0>() : (sel == 2 ? row_lines<T, NN, 2>() : row_lines<T, NN, 1>());
    PSD_FOR_EACH_N(C)
#undef C
  }
  return 0;
}
template <typename T, int NF>
int host_col_width(int n) {
  switch (n) {
#define C(NN) case NN: return col_width<T, NN, NF>();
    PSD_FOR_EACH_N(C)
#undef C
  }
  return 0;
}

}  // namespace

struct psd_handle_s {
  int batch = 0;
  int dim = 2, order = 4;
  bool p_is_4 = true;
  bool p_is_6 = false;
  bool poly_ls = true;   // p = 4 or 6: one line-search pass (polynomial q)
  psd_options opt{};
  bool mixed = false;
  hipStream_t stream = nullptr;
  bool own_stream = false;
  int device = 0;
  std::vector<psd_problem> probs;
  std::vector<Inst> hI;
  Inst* dI = nullptr;
  std::vector<Task2> hT;
  Task2* dT = nullptr;
  Range res, ls;
  FftTasks fft_solver;   // solver precision, NF of the order
  FftTasks fft_aux;      // FP64, one field (Poisson / energy / residual helpers)
  SolveState* dState = nullptr;
  SolveState* dAuxState = nullptr;  // states of auxiliary evaluations (keep dState intact)
  SolveState* hState = nullptr;  // pinned
  // graph-mode solves: two pinned slots for the states copied after each
  // queued batch of replays, each with an event (created on first use)
  SolveState* hStateQ[2] = {nullptr, nullptr};
  hipEvent_t ev_state[2] = {nullptr, nullptr};
  double* hPart = nullptr;       // pinned scratch for auxiliary partials
  size_t hPartCap = 0;
  double* dAuxPart = nullptr;
  std::vector<void*> allocs;
  hipGraphExec_t gexec = nullptr;
  hipGraph_t graph = nullptr;
  int gchunk = 0;
  bool adj_alloc = false;
  std::vector<double*> ts_f, ts_g;   // right-hand sides of the time steps (psd_timestep)
  // tuning (autotuner or defaults)
  int tune_zc_res = T3Z_RES, tune_zc_ls = T3Z_LS;
  int ls_tx = L3_TX_NARROW;   // 3D line-search tile width (wide when every n >= 64)
  int row_sel = 1;            // row-pass layout (lines per block), 0..PSD_ROW_SELS-1
  bool tune_xcd_res = false, tune_xcd_ls = false;
  size_t dT_cap = 0;
  std::string err;
  // profiling: events around every pass launch, in launch order
  struct ProfRec { int pass; int iter_slot; hipEvent_t a, b; };
  std::vector<ProfRec> prof;        // records of the current launch sequence
  std::vector<hipEvent_t> ev_pool;
  size_t ev_used = 0;
  int prof_iter_slot = -1;          // iteration index within a graph chunk (-1: none)
  double pass_ms[PSD_NPASS] = {0};
  int pass_n[PSD_NPASS] = {0};
  // arena mode (no-allocation entry point): device workspace carved from
  // `arena`, host staging in arena_hstate / arena_hpart
  char* arena = nullptr;
  size_t arena_cap = 0, arena_used = 0;
  SolveState* arena_hstate = nullptr;
  double* arena_hpart = nullptr;
};

// ---------------------------------------------------------------------------
// helpers
// ---------------------------------------------------------------------------
#define HIPCHK(expr)                                                              \
  do {                                                                            \
    hipError_t e_ = (expr);                                                       \
    if (e_ != hipSuccess) {                                                       \
      h->err = std::string(#expr) + ": " + hipGetErrorString(e_);                 \
      return PSD_ERR_HIP;                                                         \
    }                                                                             \
  } while (0)

static psd_status set_err(psd_handle* h, psd_status st, const std::string& msg) {
  if (h) h->err = msg; else g_create_error = msg;
  return st;
}

// Device workspace: hipMalloc, or 256-byte aligned pieces of the handle's
// arena (the no-allocation entry point) when one is attached.
template <typename P>
static hipError_t dalloc(psd_handle* h, P** ptr, size_t bytes) {
  if (h->arena) {
    const size_t off = (h->arena_used + 255) & ~(size_t)255;
    const size_t sz = bytes ? bytes : 16;
    if (off + sz > h->arena_cap) return hipErrorOutOfMemory;
    *ptr = (P*)(h->arena + off);
    h->arena_used = off + sz;
    return hipSuccess;
  }
  void* p = nullptr;
  hipError_t e = hipMalloc(&p, bytes ? bytes : 16);
  if (e == hipSuccess) {
    h->allocs.push_back(p);
    *ptr = (P*)p;
  }
  return e;
}

// ---------------------------------------------------------------------------
// per-pass profiling with HIP events on the solver stream
// ---------------------------------------------------------------------------
static hipEvent_t prof_event(psd_handle* h) {
  if (h->ev_used == h->ev_pool.size()) {
    hipEvent_t e;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    h->ev_pool.push_back(e);
  }
  return h->ev_pool[h->ev_used++];
}

struct ProfScope {
  psd_handle* h;
  int pass;
  hipEvent_t a = nullptr, b = nullptr;
  // Events are recorded only in host-driven (stream) mode: elapsed times of
  // events recorded through captured graph nodes are not available.
  ProfScope(psd_handle* hh, int p) : h(hh), pass(p) {
    if (!h->opt.profile || h->prof_iter_slot >= 0) pass = -1;
    if (pass < 0) return;
    a = prof_event(h);
    b = prof_event(h);
    if (a && b) (void)hipEventRecord(a, h->stream);
  }
  ~ProfScope() {
    if (!h->opt.profile || pass < 0 || !a || !b) return;
    (void)hipEventRecord(b, h->stream);
    h->prof.push_back({pass, h->prof_iter_slot, a, b});
  }
};

// Fold the recorded events into the per-pass totals (stream synchronised).
// iters_real: number of leading graph iterations that did work (-1: all).
static void prof_collect(psd_handle* h, int iters_real, bool keep_records) {
  for (const auto& r : h->prof) {
    if (iters_real >= 0 && r.iter_slot >= iters_real) continue;
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, r.a, r.b) == hipSuccess) {
      h->pass_ms[r.pass] += ms;
      h->pass_n[r.pass] += 1;
    }
  }
  if (!keep_records) { h->prof.clear(); h->ev_used = 0; }
}

extern "C" psd_status psd_check_problem(const psd_problem* prob, char* msg, int msg_len) {
  auto fail = [&](psd_status st, const char* m) {
    if (msg && msg_len > 0) { std::snprintf(msg, (size_t)msg_len, "%s", m); }
    return st;
  };
  if (!prob) return fail(PSD_ERR_ARG, "problem is NULL");
  if (prob->dim != 2 && prob->dim != 3) return fail(PSD_ERR_ARG, "dim must be 2 or 3");
  if (prob->order != 4 && prob->order != 6) return fail(PSD_ERR_ARG, "order must be 4 or 6");
  if (!n_supported(prob->n)) return fail(PSD_ERR_ARG, "unsupported n");
  if (prob->dim == 3 && (prob->n < 32 || prob->n > 256)) return fail(PSD_ERR_ARG, "3D needs 32 <= n <= 256");
  if (!(prob->L > 0.0) || !std::isfinite(prob->L)) return fail(PSD_ERR_RANGE, "L must be > 0");
  if (!(prob->s > 0.0) || !std::isfinite(prob->s)) return fail(PSD_ERR_RANGE, "s must be > 0");
  if (!(prob->eps > 0.0 && prob->eps <= 1.0)) return fail(PSD_ERR_RANGE, "eps must lie in (0, 1]");
  if (!(prob->p >= 2.0) || !std::isfinite(prob->p)) return fail(PSD_ERR_RANGE, "p must be >= 2");
  if (prob->dim == 3 && prob->p > 6.0) return fail(PSD_ERR_RANGE, "3D needs p <= 6");
  if (prob->order == 6 && !(prob->lambda >= 0.0)) return fail(PSD_ERR_RANGE, "lambda must be >= 0");
  return fail(PSD_OK, "ok");
}

// ---------------------------------------------------------------------------
// task tables
// ---------------------------------------------------------------------------
template <typename T>
static int host_cw(int n, int nf) {
  return nf == 1 ? host_col_width<T, 1>(n) : (nf == 2 ? host_col_width<T, 2>(n) : host_col_width<T, 3>(n));
}

// fs_in / fs_out: field sets read by the R2C rows and written by the C2R rows
template <typename T>
static void build_fft_tasks(psd_handle* h, FftTasks& F, int nfi, int nfo, bool with_slots, int fs_in,
                            int fs_out) {
  const size_t cxs = sizeof(cx<T>);
  F = FftTasks{};   // rebuilt after retiling: drop the previous launch groups
  // distinct transform lengths, ascending: tasks of one length are contiguous
  std::vector<int> ns;
  for (int b = 0; b < h->batch; ++b) ns.push_back(h->hI[b].n);
  std::sort(ns.begin(), ns.end());
  ns.erase(std::unique(ns.begin(), ns.end()), ns.end());
  auto open_part = [&](Range& R, int n) {
    NPart p;
    p.n = n;
    p.off = (int)h->hT.size();
    R.parts.push_back(p);
  };
  auto close_part = [&](Range& R, size_t lds) {
    NPart& p = R.parts.back();
    p.cnt = (int)h->hT.size() - p.off;
    p.lds = lds;
    R.lds = std::max(R.lds, lds);
    if (p.cnt == 0) R.parts.pop_back();
  };
  // rows R2C (nfi fields) and C2R (nfo fields)
  for (int pass = 0; pass < 2; ++pass) {
    Range& R = pass == 0 ? F.r2c : F.c2r;
    const int nf = pass == 0 ? nfi : nfo;
    R.off = (int)h->hT.size();
    for (int n : ns) {
      open_part(R, n);
      const int nl = host_row_lines<T>(n, h->row_sel);
      for (int b = 0; b < h->batch; ++b) {
        const Inst& I = h->hI[b];
        if (I.n != n) continue;
        const long long rows = (long long)nf * (I.ncell / I.n);
        int slot = 0;
        for (long long r0 = 0; r0 < rows; r0 += 2 * nl) {
          Task2 t{};
          t.inst = b; t.a = (int)r0; t.b = pass == 0 ? fs_in : fs_out; t.c = nf; t.slot = slot++;
          h->hT.push_back(t);
        }
        if (pass == 1 && with_slots) h->hI[b].nblk_c2r = slot;
      }
      close_part(R, ((size_t)nl * fft_ls(n) + n) * cxs);
    }
    R.cnt = (int)h->hT.size() - R.off;
  }
  // plain y passes (3D): forward over nfi fields, inverse over nfo fields
  for (int pass = 0; pass < 2; ++pass) {
    Range& R = pass == 0 ? F.coly_f : F.coly_i;
    const int nf = pass == 0 ? nfi : nfo;
    R.off = (int)h->hT.size();
    if (h->dim == 3) {
      for (int n : ns) {
        open_part(R, n);
        const int W = host_cw<T>(n, nf);
        for (int b = 0; b < h->batch; ++b) {
          const Inst& I = h->hI[b];
          if (I.n != n) continue;
          for (int z0 = 0; z0 < n; z0 += W) {  // Nyquist y-lines of W planes
            Task2 t{};
            t.inst = b; t.a = z0; t.c = 1;
            h->hT.push_back(t);
          }
          for (int z = 0; z < n; ++z)          // plain blocks: kx < n/2
            for (int c0 = 0; c0 < n / 2; c0 += W) {
              Task2 t{};
              t.inst = b; t.a = z; t.b = c0;
              h->hT.push_back(t);
            }
        }
        close_part(R, ((size_t)nf * W * fft_ls(n) + n) * cxs);
      }
    }
    R.cnt = (int)h->hT.size() - R.off;
  }
  // fused last-axis pass
  Range& R = F.colz;
  R.off = (int)h->hT.size();
  const int nfm = std::max(nfi, nfo);
  for (int n : ns) {
    open_part(R, n);
    const int W = host_cw<T>(n, nfm);
    for (int b = 0; b < h->batch; ++b) {
      Inst& I = h->hI[b];
      if (I.n != n) continue;
      const int rows = h->dim == 2 ? 1 : n;   // ky rows of columns (3D)
      int slot = 0;
      for (int ky0 = 0; ky0 < rows; ky0 += W) {  // Nyquist lines of W rows
        Task2 t{};
        t.inst = b; t.a = ky0; t.c = 1; t.slot = slot++;
        h->hT.push_back(t);
      }
      for (int ky = 0; ky < rows; ++ky)        // plain blocks: kx < n/2
        for (int c0 = 0; c0 < n / 2; c0 += W) {
          Task2 t{};
          t.inst = b; t.a = ky; t.b = c0; t.slot = slot++;
          h->hT.push_back(t);
        }
      if (with_slots) I.nblk_sp = slot;
    }
    close_part(R, std::max(((size_t)nfm * W * fft_ls(n) + n) * cxs + n * sizeof(double), (size_t)64 * 8));
  }
  R.cnt = (int)h->hT.size() - R.off;
}

// XCD-aware order of a launch's task list: MI355X hands workgroup i to XCD
// (i mod 8); with this permutation XCD x receives a contiguous run of the
// natural (spatial) order, so tiles that share halos share an L2.
static void xcd_permute(std::vector<Task2>& v, size_t off, size_t cnt) {
  if (cnt < 16) return;
  std::vector<Task2> nat(v.begin() + off, v.begin() + off + cnt);
  const size_t q = cnt / 8, r = cnt % 8;
  for (size_t i = 0; i < cnt; ++i) {
    const size_t x = i % 8, k = i / 8;
    const size_t start = x * q + std::min(x, r);
    v[off + i] = nat[start + k];
  }
}

static void build_tile_tasks(psd_handle* h) {
  // residual and line-search tiles: same (x, y) tiling, own z-chunk and order
  for (int pass = 0; pass < 2; ++pass) {
    Range& R = pass == 0 ? h->res : h->ls;
    const int zc = pass == 0 ? h->tune_zc_res : h->tune_zc_ls;
    const bool xcd = pass == 0 ? h->tune_xcd_res : h->tune_xcd_ls;
    R.off = (int)h->hT.size();
    for (int b = 0; b < h->batch; ++b) {
      Inst& I = h->hI[b];
      int slot = 0;
      if (h->dim == 2) {
        // residual: 64 x 8 LDS tiles; line search: 64 x 32 tiles walked by rows
        const int tyh = pass == 0 ? T2Y : L2W_Y, txw = pass == 0 ? T2X : L2W_X;
        for (int y0 = 0; y0 < I.n; y0 += tyh)
          for (int x0 = 0; x0 < I.n; x0 += txw) {
            Task2 t{}; t.inst = b; t.a = x0; t.b = y0; t.c = 0; t.slot = slot++;
            h->hT.push_back(t);
          }
      } else if (pass == 0 && h->order == 6) {
        // sixth-order residual: bricks of B6X x B6Y x B6Z cells
        for (int z0 = 0; z0 < I.n; z0 += B6Z)
          for (int y0 = 0; y0 < I.n; y0 += B6Y)
            for (int x0 = 0; x0 < I.n; x0 += B6X) {
              Task2 t{}; t.inst = b; t.a = x0; t.b = y0; t.c = z0; t.slot = slot++;
              h->hT.push_back(t);
            }
        I.zchunk_res = B6Z;
      } else {
        const int z = std::min(zc, I.n);
        const int tx = pass == 0 ? R3_TX : h->ls_tx;   // tile shape tx x ty
        const int ty = (pass == 0 ? R3_CY : L3_CY) * PSD_NT / tx;
        for (int z0 = 0; z0 < I.n; z0 += z)
          for (int y0 = 0; y0 < I.n; y0 += ty)
            for (int x0 = 0; x0 < I.n; x0 += tx) {
              Task2 t{}; t.inst = b; t.a = x0; t.b = y0; t.c = z0; t.slot = slot++;
              h->hT.push_back(t);
            }
        if (pass == 0) I.zchunk_res = z; else I.zchunk_ls = z;
      }
      if (pass == 0) I.nblk_res = slot; else I.nblk_ls = slot;
    }
    R.cnt = (int)h->hT.size() - R.off;
    if (xcd) xcd_permute(h->hT, R.off, R.cnt);
    if (h->dim == 2)
      R.lds = pass == 0 ? (R2_LDS + 16) * sizeof(double) : 32 * sizeof(double);
    else if (pass == 0 && h->order == 6)
      R.lds = (B6_LDS + 16) * sizeof(double);
    else
      R.lds = pass == 0 ? (R3Shape<R3_TX>::LDS + 16) * sizeof(double)
                        : ((h->ls_tx == L3_TX_WIDE ? L3Shape<L3_TX_WIDE>::LDS : L3Shape<L3_TX_NARROW>::LDS) + 32) *
                              sizeof(double);
  }
}

// Build every task table (tiles with the current tuning, FFT passes of the
// solver precision and the FP64 auxiliary transforms) into h->hT.
// nsp_aux[b] receives the auxiliary spectral block count of instance b.
static void build_all_tasks(psd_handle* h, std::vector<int>& nsp_aux) {
  h->hT.clear();
  build_tile_tasks(h);
  const int nfi = h->order == 6 ? 2 : 1, nfo = h->order == 6 ? 3 : 1;
  if (h->mixed) build_fft_tasks<float>(h, h->fft_solver, nfi, nfo, true, FS_RES, FS_DIR);
  else build_fft_tasks<double>(h, h->fft_solver, nfi, nfo, true, FS_RES, FS_DIR);
  build_fft_tasks<double>(h, h->fft_aux, 1, 1, false, FS_TMP, FS_TMP);
  nsp_aux.assign(h->batch, 0);
  for (int k = 0; k < h->fft_aux.colz.cnt; ++k) {
    Task2& t = h->hT[h->fft_aux.colz.off + k];
    t.slot = nsp_aux[t.inst]++;
  }
}

// ---------------------------------------------------------------------------
// launches
// ---------------------------------------------------------------------------
// One launch per pass: the kernel specialised to the transform length when
// the batch has one grid size, else the kernel that switches per block.
template <typename T, typename TIO, bool FWD, int SEL>
static void launch_rows_sel(const Range& R, const Inst* dI, const Task2* dT, int sv, hipStream_t s) {
  if (R.parts.size() > 1) {
    k_rows_any<T, TIO, FWD, SEL><<<R.cnt, PSD_NT, R.lds, s>>>(dI, dT + R.off, sv);
    return;
  }
  for (const NPart& p : R.parts) {
    switch (p.n) {
#define PSD_L(NN) \
      case NN: k_rows<T, TIO, FWD, NN, SEL><<<p.cnt, PSD_NT, p.lds, s>>>(dI, dT + p.off, sv); break;
      PSD_FOR_EACH_N(PSD_L)
#undef PSD_L
      default: break;
    }
  }
}

// row-pass layout `sel` (lines per block, see row_lines) as built into the tasks
template <typename T, typename TIO, bool FWD>
static void launch_rows(const Range& R, const Inst* dI, const Task2* dT, int sv, hipStream_t s, int sel) {
  if (sel == 0) launch_rows_sel<T, TIO, FWD, 0>(R, dI, dT, sv, s);
  else if (sel == 2) launch_rows_sel<T, TIO, FWD, 2>(R, dI, dT, sv, s);
  else launch_rows_sel<T, TIO, FWD, 1>(R, dI, dT, sv, s);
}

template <typename T, int NF, int DIR>
static void launch_cols(const Range& R, const Inst* dI, const Task2* dT, int sv, hipStream_t s) {
  if (R.parts.size() > 1) {
    k_cols_any<T, NF, DIR><<<R.cnt, PSD_NT, R.lds, s>>>(dI, dT + R.off, sv);
    return;
  }
  for (const NPart& p : R.parts) {
    switch (p.n) {
#define PSD_L(NN) \
      case NN: k_cols<T, NF, DIR, NN><<<p.cnt, PSD_NT, p.lds, s>>>(dI, dT + p.off, sv); break;
      PSD_FOR_EACH_N3(PSD_L)
#undef PSD_L
      default: break;
    }
  }
}

template <typename T, int OP>
static void launch_fused(const Range& R, const Inst* dI, const Task2* dT, int sv, hipStream_t s) {
  if (R.parts.size() > 1) {
    k_cols_fused_any<T, OP><<<R.cnt, PSD_NT, R.lds, s>>>(dI, dT + R.off, sv);
    return;
  }
  for (const NPart& p : R.parts) {
    switch (p.n) {
#define PSD_L(NN) \
      case NN: k_cols_fused<T, OP, NN><<<p.cnt, PSD_NT, p.lds, s>>>(dI, dT + p.off, sv); break;
      PSD_FOR_EACH_N(PSD_L)
#undef PSD_L
      default: break;
    }
  }
}

template <typename T, typename TIN, typename TOUT>
static void run_fft(psd_handle* h, const FftTasks& F, int op, bool solver) {
  const Task2* dT = h->dT;
  const Inst* dI = h->dI;
  hipStream_t s = h->stream;
  const int sv = solver ? 1 : 0;
  const bool pr = solver;  // auxiliary transforms are not profiled
  if (F.r2c.cnt) {
    ProfScope ps(h, pr ? PSD_PASS_ROWS_R2C : -1);
    launch_rows<T, TIN, true>(F.r2c, dI, dT, sv, s, h->row_sel);
  }
  const int nfi = op == OP_PRECOND6 ? 2 : 1, nfo = op == OP_PRECOND6 ? 3 : 1;
  if (F.coly_f.cnt) {
    ProfScope ps(h, pr ? PSD_PASS_COLS_FWD : -1);
    if (nfi == 1) launch_cols<T, 1, -1>(F.coly_f, dI, dT, sv, s);
    else launch_cols<T, 2, -1>(F.coly_f, dI, dT, sv, s);
  }
  {
    ProfScope ps(h, pr ? PSD_PASS_COLS_FUSED : -1);
    if (op == OP_PRECOND4) launch_fused<T, OP_PRECOND4>(F.colz, dI, dT, sv, s);
    else if (op == OP_PRECOND6) launch_fused<T, OP_PRECOND6>(F.colz, dI, dT, sv, s);
    else if (op == OP_PRECOND6S) launch_fused<T, OP_PRECOND6S>(F.colz, dI, dT, sv, s);
    else launch_fused<T, OP_POISSON>(F.colz, dI, dT, sv, s);
  }
  if (F.coly_i.cnt) {
    ProfScope ps(h, pr ? PSD_PASS_COLS_INV : -1);
    if (nfo == 1) launch_cols<T, 1, 1>(F.coly_i, dI, dT, sv, s);
    else launch_cols<T, 3, 1>(F.coly_i, dI, dT, sv, s);
  }
  if (F.c2r.cnt) {
    ProfScope ps(h, pr ? PSD_PASS_ROWS_C2R : -1);
    launch_rows<T, TOUT, false>(F.c2r, dI, dT, sv, s, h->row_sel);
  }
}

template <typename TD, typename TR, int TX>
static void launch_res3d(int pk, bool upd, int n, size_t lds, hipStream_t s, const Inst* dI, const Task2* t) {
  if (pk == 4) {
    if (upd) k_res3d<TD, TR, true, 4, TX><<<n, PSD_NT, lds, s>>>(dI, t);
    else k_res3d<TD, TR, false, 4, TX><<<n, PSD_NT, lds, s>>>(dI, t);
  } else if (pk == 2) {
    if (upd) k_res3d<TD, TR, true, 2, TX><<<n, PSD_NT, lds, s>>>(dI, t);
    else k_res3d<TD, TR, false, 2, TX><<<n, PSD_NT, lds, s>>>(dI, t);
  } else if (pk == 6) {
    if (upd) k_res3d<TD, TR, true, 6, TX><<<n, PSD_NT, lds, s>>>(dI, t);
    else k_res3d<TD, TR, false, 6, TX><<<n, PSD_NT, lds, s>>>(dI, t);
  } else {
    if (upd) k_res3d<TD, TR, true, 0, TX><<<n, PSD_NT, lds, s>>>(dI, t);
    else k_res3d<TD, TR, false, 0, TX><<<n, PSD_NT, lds, s>>>(dI, t);
  }
}

template <typename TD, typename TR>
static void run_residual(psd_handle* h, bool upd) {
  hipStream_t s = h->stream;
  const Task2* t = h->dT + h->res.off;
  const int n = h->res.cnt;
  {
    ProfScope ps(h, upd ? PSD_PASS_RES : -1);
    if (h->dim == 2) {
      if (h->order == 4) {
        if (upd) k_res2d<TD, TR, 4, true><<<n, PSD_NT, h->res.lds, s>>>(h->dI, t);
        else k_res2d<TD, TR, 4, false><<<n, PSD_NT, h->res.lds, s>>>(h->dI, t);
      } else {
        if (upd) k_res2d<TD, TR, 6, true><<<n, PSD_NT, h->res.lds, s>>>(h->dI, t);
        else k_res2d<TD, TR, 6, false><<<n, PSD_NT, h->res.lds, s>>>(h->dI, t);
      }
    } else if (h->order == 6) {
      if (upd) k_res3d6<TD, TR, true><<<n, PSD_NT, h->res.lds, s>>>(h->dI, t);
      else k_res3d6<TD, TR, false><<<n, PSD_NT, h->res.lds, s>>>(h->dI, t);
    } else {
      // exponent class of the flux (all instances share p) and tile width
      const double p = h->hI[0].p;
      const int pk = p == 4.0 ? 4 : (p == 2.0 ? 2 : (p == 6.0 ? 6 : 0));
      launch_res3d<TD, TR, R3_TX>(pk, upd, n, h->res.lds, s, h->dI, t);
    }
  }
  ProfScope ps(h, upd ? PSD_PASS_RES_FIN : -1);
  k_res_finalize<<<h->batch, PSD_FIN_NT, 0, s>>>(h->dI, upd ? 1 : 0);
}

// evaluation passes of the general-p root search captured per iteration in
// graph mode (the search typically needs two to four)
constexpr int PSD_LS_GRAPH_EVALS = 6;
constexpr int PSD_LS_HOST_EVALS = 100;

template <typename TD>
static void run_ls(psd_handle* h, int mode, int max_evals = PSD_LS_HOST_EVALS) {
  hipStream_t s = h->stream;
  const Task2* t = h->dT + h->ls.off;
  {
    ProfScope ps(h, PSD_PASS_LS);
    const int nb = h->ls.cnt;
    const size_t lds = h->ls.lds;
    if (h->dim == 2) {
      if (mode == 0) k_ls2d<TD, 0><<<nb, PSD_NT, lds, s>>>(h->dI, t);
      else if (mode == 1) k_ls2d<TD, 1><<<nb, PSD_NT, lds, s>>>(h->dI, t);
      else if (mode == 3) k_ls2d<TD, 3><<<nb, PSD_NT, lds, s>>>(h->dI, t);
      else k_ls2d<TD, 2><<<nb, PSD_NT, lds, s>>>(h->dI, t);
    } else {
      if (h->ls_tx == L3_TX_WIDE) {
        if (mode == 0) k_ls3d<TD, 0, L3_TX_WIDE><<<nb, PSD_NT, lds, s>>>(h->dI, t);
        else if (mode == 1) k_ls3d<TD, 1, L3_TX_WIDE><<<nb, PSD_NT, lds, s>>>(h->dI, t);
        else if (mode == 3) k_ls3d<TD, 3, L3_TX_WIDE><<<nb, PSD_NT, lds, s>>>(h->dI, t);
        else k_ls3d<TD, 2, L3_TX_WIDE><<<nb, PSD_NT, lds, s>>>(h->dI, t);
      } else {
        if (mode == 0) k_ls3d<TD, 0, L3_TX_NARROW><<<nb, PSD_NT, lds, s>>>(h->dI, t);
        else if (mode == 1) k_ls3d<TD, 1, L3_TX_NARROW><<<nb, PSD_NT, lds, s>>>(h->dI, t);
        else if (mode == 3) k_ls3d<TD, 3, L3_TX_NARROW><<<nb, PSD_NT, lds, s>>>(h->dI, t);
        else k_ls3d<TD, 2, L3_TX_NARROW><<<nb, PSD_NT, lds, s>>>(h->dI, t);
      }
    }
  }
  ProfScope ps(h, PSD_PASS_LS_FIN);
  k_ls_finalize<<<h->batch, PSD_FIN_NT, 0, s>>>(h->dI, mode, max_evals);
}

// one PSD iteration with a polynomial q (p = 4 cubic, p = 6 quintic; Sec.
// 6.1): a fixed launch sequence, capturable in a graph
template <typename T, typename TD, typename TR>
static void run_iteration_poly(psd_handle* h) {
  run_fft<T, TR, TD>(h, h->fft_solver, h->order == 4 ? OP_PRECOND4 : OP_PRECOND6, true);
  run_ls<TD>(h, h->p_is_6 ? 3 : 0);
  run_residual<TD, TR>(h, true);
}

// Copy the states the instance table currently points at (the solver's, or
// the auxiliary ones) to the host.
static psd_status read_states(psd_handle* h) {
  HIPCHK(hipMemcpyAsync(h->hState, h->hI[0].st, sizeof(SolveState) * h->batch, hipMemcpyDeviceToHost,
                        h->stream));
  HIPCHK(hipStreamSynchronize(h->stream));
  return PSD_OK;
}

static bool all_done(psd_handle* h) {
  for (int b = 0; b < h->batch; ++b)
    if (!h->hState[b].done) return false;
  return true;
}

// general p, host-driven loop: the host polls the root search after every
// evaluation pass (one grid pass per evaluation of q and q')
template <typename TD>
static psd_status run_ls_general(psd_handle* h) {
  run_ls<TD>(h, 1);
  for (int step = 0; step < PSD_LS_HOST_EVALS; ++step) {
    run_ls<TD>(h, 2);
    psd_status st = read_states(h);
    if (st != PSD_OK) return st;
    bool fin = true;
    for (int b = 0; b < h->batch; ++b)
      if (!h->hState[b].done && h->hState[b].ls_phase != 2) fin = false;
    if (fin) break;
  }
  return PSD_OK;
}

template <typename T, typename TD, typename TR>
static psd_status run_iteration_general(psd_handle* h) {
  run_fft<T, TR, TD>(h, h->fft_solver, h->order == 4 ? OP_PRECOND4 : OP_PRECOND6, true);
  psd_status st = run_ls_general<TD>(h);
  if (st != PSD_OK) return st;
  run_residual<TD, TR>(h, true);
  return PSD_OK;
}

// general p, graph mode: a fixed number of evaluation passes; the blocks of
// passes after the search has finished return at once
template <typename T, typename TD, typename TR>
static void run_iteration_general_fixed(psd_handle* h) {
  run_fft<T, TR, TD>(h, h->fft_solver, h->order == 4 ? OP_PRECOND4 : OP_PRECOND6, true);
  run_ls<TD>(h, 1);
  for (int step = 0; step < PSD_LS_GRAPH_EVALS; ++step) run_ls<TD>(h, 2, PSD_LS_GRAPH_EVALS);
  run_residual<TD, TR>(h, true);
}

// search direction of the variable metric (defined with the adjoint's
// conjugate-gradient machinery below)
template <typename T, typename TD, typename TR>
static psd_status vm_direction(psd_handle* h);

template <typename T, typename TD, typename TR>
static psd_status solve_loop(psd_handle* h) {
  const int chunk = h->opt.graph_chunk;
  if (chunk > 0 && h->opt.metric != PSD_METRIC_VARIABLE) {
    if (!h->gexec || h->gchunk != chunk) {
      if (h->gexec) { (void)hipGraphExecDestroy(h->gexec); h->gexec = nullptr; }
      if (h->graph) { (void)hipGraphDestroy(h->graph); h->graph = nullptr; }
      h->prof.clear();
      h->ev_used = 0;
      HIPCHK(hipStreamBeginCapture(h->stream, hipStreamCaptureModeThreadLocal));
      for (int k = 0; k < chunk; ++k) {
        h->prof_iter_slot = k;
        if (h->poly_ls) run_iteration_poly<T, TD, TR>(h);
        else run_iteration_general_fixed<T, TD, TR>(h);
      }
      h->prof_iter_slot = -1;
      HIPCHK(hipStreamEndCapture(h->stream, &h->graph));
      HIPCHK(hipGraphInstantiate(&h->gexec, h->graph, nullptr, nullptr, 0));
      h->gchunk = chunk;
    }
    // Replays are queued in batches.  After the initial residual and after
    // each batch the device states are copied to a pinned slot and an event
    // is recorded; the host queues the next batch before it waits for the
    // previous one's states, so the GPU does not idle while the host decides
    // (at most two batches are outstanding).  The batch size comes from the
    // residual decay observed so far (PSD converges linearly, Sec. 2.3):
    // enough replays to reach tol at the measured rate counting those already
    // queued.  Replays past convergence cost only early exits.
    for (int k = 0; k < 2; ++k) {
      if (!h->hStateQ[k] &&
          hipHostMalloc((void**)&h->hStateQ[k], sizeof(SolveState) * h->batch, hipHostMallocDefault) != hipSuccess)
        return set_err(h, PSD_ERR_HIP, "pinned allocation failed");
      if (!h->ev_state[k] && hipEventCreateWithFlags(&h->ev_state[k], hipEventDisableTiming) != hipSuccess)
        return set_err(h, PSD_ERR_HIP, "event creation failed");
    }
    const int max_launch = h->opt.max_iter / chunk + 2;
    struct Batch { int slot, chunks; };
    Batch q[2];
    int nq = 0, next_slot = 0, launched = 0;
    auto enqueue = [&](int nrep) -> psd_status {
      int c = 0;
      for (; c < nrep && launched < max_launch; ++c, ++launched) HIPCHK(hipGraphLaunch(h->gexec, h->stream));
      const int sl = next_slot;
      next_slot ^= 1;
      HIPCHK(hipMemcpyAsync(h->hStateQ[sl], h->hI[0].st, sizeof(SolveState) * h->batch, hipMemcpyDeviceToHost,
                            h->stream));
      HIPCHK(hipEventRecord(h->ev_state[sl], h->stream));
      q[nq++] = Batch{sl, c};
      return PSD_OK;
    };
    psd_status st = enqueue(0);   // the initial residual's states
    if (st == PSD_OK) st = enqueue(1);
    if (st != PSD_OK) return st;
    std::vector<double> r_prev(h->batch, 0.0);
    std::vector<int> k_prev(h->batch, -1);
    while (nq > 0) {
      const Batch bt = q[0];
      q[0] = q[1];
      --nq;
      HIPCHK(hipEventSynchronize(h->ev_state[bt.slot]));
      const SolveState* S = h->hStateQ[bt.slot];
      bool done = true, rate_known = true;
      double k_rem = 0.0;
      for (int b = 0; b < h->batch; ++b) {
        if (S[b].done) continue;
        done = false;
        const int dk = k_prev[b] < 0 ? 0 : S[b].iter - k_prev[b];
        double need = chunk;
        if (dk > 0 && S[b].rinf > 0.0 && r_prev[b] > S[b].rinf) {
          const double rate = std::pow(S[b].rinf / r_prev[b], 1.0 / dk);   // per iteration
          need = std::log(h->hI[b].tol / S[b].rinf) / std::log(rate);
        } else {
          rate_known = false;
        }
        k_rem = std::max(k_rem, need);
        r_prev[b] = S[b].rinf;
        k_prev[b] = S[b].iter;
      }
      if (done) break;
      int ahead = 0;   // replays still queued
      for (int k = 0; k < nq; ++k) ahead += q[k].chunks;
      int nrep = (int)std::ceil((std::min(k_rem, (double)h->opt.max_iter) - ahead * chunk) / chunk);
      nrep = std::max(0, std::min(nrep, 8));
      if (nq == 0 || !rate_known) nrep = std::max(nrep, 1);
      if (nrep > 0 && launched < max_launch) {
        st = enqueue(nrep);
        if (st != PSD_OK) return st;
      }
    }
    return PSD_OK;
  }
  for (int it = 0; it <= h->opt.max_iter; ++it) {
    if (h->opt.metric == PSD_METRIC_VARIABLE) {
      psd_status st = vm_direction<T, TD, TR>(h);
      if (st != PSD_OK) return st;
      if (h->poly_ls) run_ls<TD>(h, h->p_is_6 ? 3 : 0);
      else {
        st = run_ls_general<TD>(h);
        if (st != PSD_OK) return st;
      }
      run_residual<TD, TR>(h, true);
    } else if (h->poly_ls) {
      run_iteration_poly<T, TD, TR>(h);
    } else {
      psd_status st = run_iteration_general<T, TD, TR>(h);
      if (st != PSD_OK) return st;
    }
    HIPCHK(hipGetLastError());
    psd_status st = read_states(h);
    if (st != PSD_OK) return st;
    if (h->opt.profile) prof_collect(h, -1, false);
    if (all_done(h)) break;
  }
  return PSD_OK;
}

// sum of per-block auxiliary partials on the host (fixed order)
static psd_status aux_sums(psd_handle* h, const double* a, const double* b, long long N, double out[3]) {
  const int nblk = 256;
  k_sums<<<nblk, PSD_NT, 0, h->stream>>>(a, b, N, h->dAuxPart);
  HIPCHK(hipGetLastError());
  HIPCHK(hipMemcpyAsync(h->hPart, h->dAuxPart, sizeof(double) * 3 * nblk, hipMemcpyDeviceToHost, h->stream));
  HIPCHK(hipStreamSynchronize(h->stream));
  out[0] = out[1] = out[2] = 0.0;
  for (int k = 0; k < nblk; ++k)
    for (int q = 0; q < 3; ++q) out[q] += h->hPart[3 * k + q];
  return PSD_OK;
}

static psd_status upload_inst(psd_handle* h) {
  HIPCHK(hipMemcpyAsync(h->dI, h->hI.data(), sizeof(Inst) * h->batch, hipMemcpyHostToDevice, h->stream));
  return PSD_OK;
}

// Apply T_h = -Delta_h^{-1} (FP64) to I.tmp of instance b in place; returns
// sum_k w |z^|^2/K / Ntot = (z, T_h z) without the h^dim factor.
static psd_status aux_poisson(psd_handle* h, int b, double* zTz) {
  // run the auxiliary FFT only on instance b: temporarily mark the others done
  run_fft<double, double, double>(h, h->fft_aux, OP_POISSON, false);
  HIPCHK(hipGetLastError());
  if (zTz) {
    const Inst& I = h->hI[b];
    // partials live in part_sp of instance b (aux slot count = fft_aux blocks of b)
    int nblk = 0;
    for (int k = 0; k < h->fft_aux.colz.cnt; ++k)
      if (h->hT[h->fft_aux.colz.off + k].inst == b) ++nblk;
    std::vector<double> tmp(2 * (size_t)nblk);
    HIPCHK(hipMemcpyAsync(tmp.data(), I.part_sp, sizeof(double) * 2 * nblk, hipMemcpyDeviceToHost, h->stream));
    HIPCHK(hipStreamSynchronize(h->stream));
    double sacc = 0.0;
    for (int k = 0; k < nblk; ++k) sacc += tmp[2 * k];
    *zTz = sacc;
  }
  return PSD_OK;
}

// ---------------------------------------------------------------------------
// autotuner: stencil tilings timed on the handle's own buffers
// ---------------------------------------------------------------------------
static std::string tune_key(psd_handle* h) {
  hipDeviceProp_t prop;
  std::string arch = "gfx";
  if (hipGetDeviceProperties(&prop, h->device) == hipSuccess) arch = prop.gcnArchName;
  std::string k = arch + " d" + std::to_string(h->dim) + " o" + std::to_string(h->order) +
                  (h->mixed ? " mixed" : " fp64") + " n";
  for (int b = 0; b < h->batch; ++b) k += (b ? "," : "") + std::to_string(h->hI[b].n);
  if (k.size() > 200) k = k.substr(0, 200) + " b" + std::to_string(h->batch);
  return k;
}

static bool tune_cache_read(psd_handle* h, const std::string& key) {
  const char* path = std::getenv("PSD_TUNE_CACHE");
  if (!path) return false;
  FILE* fp = std::fopen(path, "r");
  if (!fp) return false;
  char line[512];
  bool found = false;
  while (std::fgets(line, sizeof line, fp)) {
    std::string l(line);
    const size_t bar = l.find('|');
    if (bar == std::string::npos || l.substr(0, bar) != key) continue;
    int a, b, c, d, e, rs = 1;
    // chunks below T3Z_MIN would need more partial slots than were allocated;
    // a wide line-search tile needs every n >= 64; the row layout is the
    // sixth value (lines without it keep the default layout)
    const int nv = std::sscanf(l.c_str() + bar + 1, "%d %d %d %d %d %d", &a, &b, &c, &d, &e, &rs);
    if (nv >= 5 && a >= T3Z_MIN && b >= T3Z_MIN && (e == L3_TX_NARROW || (e == L3_TX_WIDE && h->ls_tx == L3_TX_WIDE)) &&
        rs >= 0 && rs < PSD_ROW_SELS) {
      h->tune_zc_res = a; h->tune_zc_ls = b; h->tune_xcd_res = c != 0; h->tune_xcd_ls = d != 0;
      h->ls_tx = e;
      h->row_sel = rs;
      found = true;
    }
  }
  std::fclose(fp);
  return found;
}

static void tune_cache_write(psd_handle* h, const std::string& key) {
  const char* path = std::getenv("PSD_TUNE_CACHE");
  if (!path) return;
  FILE* fp = std::fopen(path, "a");
  if (!fp) return;
  std::fprintf(fp, "%s|%d %d %d %d %d %d\n", key.c_str(), h->tune_zc_res, h->tune_zc_ls, (int)h->tune_xcd_res,
               (int)h->tune_xcd_ls, h->ls_tx, h->row_sel);
  std::fclose(fp);
}

static psd_status upload_tasks(psd_handle* h) {
  if (h->hT.size() > h->dT_cap) return set_err(h, PSD_ERR_ARG, "task table exceeds its capacity");
  HIPCHK(hipMemcpyAsync(h->dT, h->hT.data(), sizeof(Task2) * h->hT.size(), hipMemcpyHostToDevice, h->stream));
  HIPCHK(hipMemcpyAsync(h->dI, h->hI.data(), sizeof(Inst) * h->batch, hipMemcpyHostToDevice, h->stream));
  HIPCHK(hipStreamSynchronize(h->stream));
  return PSD_OK;
}

// timed repetitions per autotuner candidate (after one warm-up) and the
// margin by which another row layout must beat the default one
constexpr int PSD_TUNE_REPS = 5;
constexpr double PSD_TUNE_MARGIN = 0.03;

static double median_of(std::vector<double> v) {
  if (v.empty()) return 0.0;
  std::sort(v.begin(), v.end());
  const size_t m = v.size() / 2;
  return v.size() % 2 ? v[m] : 0.5 * (v[m - 1] + v[m]);
}

template <typename TD, typename TR>
static psd_status autotune_impl(psd_handle* h) {
  const std::string key = tune_key(h);
  std::vector<int> nsp_aux;
  if (tune_cache_read(h, key)) {
    build_all_tasks(h, nsp_aux);
    return upload_tasks(h);
  }
  // scratch bindings: u[0] -> tmp, f -> u[1] (a buffer of its own, as in a
  // solve; every residual block reads f only at the cells whose new iterate
  // it writes, and both stay zero); d, r zeroed
  std::vector<Inst> saved = h->hI;
  for (int b = 0; b < h->batch; ++b) {
    Inst& I = h->hI[b];
    const size_t tds = h->mixed ? 4 : 8;
    HIPCHK(hipMemsetAsync(I.tmp, 0, I.ncell * 8, h->stream));
    HIPCHK(hipMemsetAsync(I.d, 0, I.ncell * tds, h->stream));
    HIPCHK(hipMemsetAsync(I.r, 0, I.ncell * tds, h->stream));
    HIPCHK(hipMemsetAsync(I.u[1], 0, I.ncell * 8, h->stream));
    if (h->order == 6) HIPCHK(hipMemsetAsync(I.r1, 0, I.ncell * tds, h->stream));
    I.u[0] = I.tmp;
    I.f = I.u[1];
    if (h->order == 6) {
      HIPCHK(hipMemsetAsync(I.w[0], 0, I.ncell * 8, h->stream));
      HIPCHK(hipMemsetAsync(I.w[1], 0, I.ncell * 8, h->stream));
      HIPCHK(hipMemsetAsync(I.e1, 0, I.ncell * (h->mixed ? 4 : 8), h->stream));
      HIPCHK(hipMemsetAsync(I.e2, 0, I.ncell * (h->mixed ? 4 : 8), h->stream));
      I.g = I.tmp;
    }
  }
  // z-chunk candidates (residual, line search): whole groups of six steps
  std::vector<int> zres = {16, 28, 40, 64}, zls = {12, 24, 36, 60};
  if (h->dim == 2) { zres = {T3Z_RES}; zls = {T3Z_LS}; }
  else {
    // plus the chunk at which the whole grid is one round of resident blocks
    // (column tiles x chunks = CUs x blocks per CU), rounded up to whole groups
    // of six steps: no block waits for a slot and no slot idles at the end
    int ncu = 256;
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, h->device) == hipSuccess) ncu = prop.multiProcessorCount;
    int occ_res = 0, occ_ls = 0;
    const size_t lds_ls = ((h->ls_tx == L3_TX_WIDE ? L3Shape<L3_TX_WIDE>::LDS : L3Shape<L3_TX_NARROW>::LDS) + 32) *
                          sizeof(double);
    HIPCHK(hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ_res, k_res3d<TD, TR, true, 4, R3_TX>, PSD_NT,
                                                        (R3Shape<R3_TX>::LDS + 16) * sizeof(double)));
    if (h->ls_tx == L3_TX_WIDE)
      HIPCHK(hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ_ls, k_ls3d<TD, 0, L3_TX_WIDE>, PSD_NT, lds_ls));
    else
      HIPCHK(hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ_ls, k_ls3d<TD, 0, L3_TX_NARROW>, PSD_NT, lds_ls));
    auto balanced = [&](int tx, int ty, int occ, int extra_steps) {
      long long tiles = 0;
      int nmax = 0;
      for (int b = 0; b < h->batch; ++b) {
        const int n = h->hI[b].n;
        tiles += (long long)((n + tx - 1) / tx) * ((n + ty - 1) / ty);
        nmax = std::max(nmax, n);
      }
      const long long k = std::max(1LL, (long long)ncu * std::max(occ, 1) / std::max(tiles, 1LL));
      int z = std::max((int)((nmax + k - 1) / k), T3Z_MIN);
      while ((z + extra_steps) % 6) ++z;
      return z;
    };
    const int zr = balanced(R3_TX, R3_CY * PSD_NT / R3_TX, occ_res, 2);
    const int zl = balanced(h->ls_tx, L3_CY * PSD_NT / h->ls_tx, occ_ls, 0);
    bool seen = false;
    for (size_t i = 0; i < zres.size(); ++i) seen = seen || (zres[i] == zr && zls[i] == zl);
    if (!seen) { zres.push_back(zr); zls.push_back(zl); }
  }
  const int save_prof = h->opt.profile;
  h->opt.profile = 1;
  double best_res = 1e300, best_ls = 1e300;
  int bz_res = T3Z_RES, bz_ls = T3Z_LS;
  bool bx_res = false, bx_ls = false;
  // line-search tile widths: 64 only where every grid has n >= 64
  std::vector<int> txs = {h->ls_tx};
  if (h->dim == 3 && h->ls_tx == L3_TX_WIDE) txs.push_back(L3_TX_NARROW);
  int btx_ls = h->ls_tx;
  for (size_t zi = 0; zi < zres.size(); ++zi)
  for (int tx : txs) {
    for (int xcd = 0; xcd < 2; ++xcd) {
      h->ls_tx = tx;
      h->tune_zc_res = zres[zi];
      h->tune_zc_ls = zls[zi];
      h->tune_xcd_res = h->tune_xcd_ls = xcd != 0;
      build_all_tasks(h, nsp_aux);
      psd_status st = upload_tasks(h);
      if (st != PSD_OK) return st;
      // the launch sequence of an iteration (the transforms leave the caches
      // as they are when the line search starts); stencil passes timed, the
      // median over the timed repetitions kept
      std::vector<double> vr, vl;
      for (int rep = 0; rep < 1 + PSD_TUNE_REPS; ++rep) {
        for (int k = 0; k < PSD_NPASS; ++k) { h->pass_ms[k] = 0.0; h->pass_n[k] = 0; }
        k_reset_state<<<(h->batch + 63) / 64, 64, 0, h->stream>>>(h->dI, h->batch);
        run_fft<TD, TR, TD>(h, h->fft_solver, h->order == 4 ? OP_PRECOND4 : OP_PRECOND6, true);
        run_ls<TD>(h, 0);
        k_reset_state<<<(h->batch + 63) / 64, 64, 0, h->stream>>>(h->dI, h->batch);
        run_residual<TD, TR>(h, true);
        HIPCHK(hipStreamSynchronize(h->stream));
        if (rep == 0) { h->prof.clear(); h->ev_used = 0; continue; }  // warm-up
        prof_collect(h, -1, false);
        vr.push_back(h->pass_ms[PSD_PASS_RES]);
        vl.push_back(h->pass_ms[PSD_PASS_LS]);
      }
      HIPCHK(hipGetLastError());
      const double tr = median_of(vr), tl = median_of(vl);
      if (tr < best_res) { best_res = tr; bz_res = zres[zi]; bx_res = xcd != 0; }
      if (tl < best_ls) { best_ls = tl; bz_ls = zls[zi]; bx_ls = xcd != 0; btx_ls = tx; }
    }
  }
  h->tune_zc_res = bz_res; h->tune_zc_ls = bz_ls;
  h->tune_xcd_res = bx_res; h->tune_xcd_ls = bx_ls;
  h->ls_tx = btx_ls;
  // row-pass layout (lines per block of the LDS row transform): both row
  // passes of the solver's transform timed for every layout
  double best_rows = 1e300, rows_ms[PSD_ROW_SELS] = {0.0, 0.0, 0.0};
  int bsel = 1;
  for (int sel = 0; sel < PSD_ROW_SELS; ++sel) {
    h->row_sel = sel;
    build_all_tasks(h, nsp_aux);
    psd_status st = upload_tasks(h);
    if (st != PSD_OK) return st;
    std::vector<double> vt;
    for (int rep = 0; rep < 1 + PSD_TUNE_REPS; ++rep) {
      for (int k = 0; k < PSD_NPASS; ++k) { h->pass_ms[k] = 0.0; h->pass_n[k] = 0; }
      k_reset_state<<<(h->batch + 63) / 64, 64, 0, h->stream>>>(h->dI, h->batch);
      run_fft<TD, TR, TD>(h, h->fft_solver, h->order == 4 ? OP_PRECOND4 : OP_PRECOND6, true);
      HIPCHK(hipStreamSynchronize(h->stream));
      if (rep == 0) { h->prof.clear(); h->ev_used = 0; continue; }  // warm-up
      prof_collect(h, -1, false);
      vt.push_back(h->pass_ms[PSD_PASS_ROWS_R2C] + h->pass_ms[PSD_PASS_ROWS_C2R]);
    }
    HIPCHK(hipGetLastError());
    const double trow = median_of(vt);
    rows_ms[sel] = trow;
    if (trow < best_rows) { best_rows = trow; bsel = sel; }
  }
  // the default layout unless another one is clearly faster (the timings of
  // near-equal layouts swap from run to run)
  if (bsel != 1 && rows_ms[1] <= best_rows * (1.0 + PSD_TUNE_MARGIN)) bsel = 1;
  h->row_sel = bsel;
  h->opt.profile = save_prof;
  h->hI = saved;
  build_all_tasks(h, nsp_aux);
  for (int k = 0; k < PSD_NPASS; ++k) { h->pass_ms[k] = 0.0; h->pass_n[k] = 0; }
  psd_status st = upload_tasks(h);
  if (st != PSD_OK) return st;
  HIPCHK(hipMemsetAsync(h->dState, 0, sizeof(SolveState) * h->batch, h->stream));
  HIPCHK(hipStreamSynchronize(h->stream));
  tune_cache_write(h, key);
  return PSD_OK;
}

// ---------------------------------------------------------------------------
// C ABI
// ---------------------------------------------------------------------------
// Validate a problem batch and options (host only).
static psd_status check_create_args(const psd_problem* probs, int batch, const psd_options* opt,
                                    std::string& msg_out) {
  if (!probs || batch <= 0 || !opt) { msg_out = "probs/opt NULL or batch <= 0"; return PSD_ERR_ARG; }
  char msg[128];
  for (int b = 0; b < batch; ++b) {
    psd_status st = psd_check_problem(&probs[b], msg, sizeof msg);
    if (st != PSD_OK) { msg_out = "instance " + std::to_string(b) + ": " + msg; return st; }
    if (probs[b].dim != probs[0].dim || probs[b].order != probs[0].order || probs[b].p != probs[0].p) {
      msg_out = "all instances must share dim, order and p";
      return PSD_ERR_ARG;
    }
  }
  if (!(opt->tol >= 0.0) || opt->max_iter < 0 || (opt->precision != PSD_FP64 && opt->precision != PSD_MIXED) ||
      opt->graph_chunk < 0) {
    msg_out = "bad options";
    return PSD_ERR_ARG;
  }
  if (opt->metric != PSD_METRIC_CONSTANT && opt->metric != PSD_METRIC_VARIABLE) {
    msg_out = "metric must be PSD_METRIC_CONSTANT or PSD_METRIC_VARIABLE";
    return PSD_ERR_ARG;
  }
  if (opt->metric == PSD_METRIC_VARIABLE &&
      (probs[0].order != 4 || opt->graph_chunk != 0 || opt->inner_iters < 1 || !(opt->inner_rtol >= 0.0))) {
    msg_out = "the variable metric needs order 4, graph_chunk 0, inner_iters >= 1 and inner_rtol >= 0";
    return PSD_ERR_ARG;
  }
  return PSD_OK;
}

__global__ void k_fill_zero(double* __restrict__ p, long long n) {
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x)
    p[i] = 0.0;
}

// Workspace, tables and task lists of a handle whose batch, options and
// stream are set.  Device memory comes from dalloc (hipMalloc, or the handle's
// arena when one is attached); host staging of the solver state is pinned
// memory, or the arena's host buffers.  On failure h->err holds the reason.
static psd_status setup_handle(psd_handle* h, const psd_problem* probs, int batch, const psd_options* opt) {
  h->batch = batch;
  h->dim = probs[0].dim;
  h->order = probs[0].order;
  h->p_is_4 = probs[0].p == 4.0;
  h->p_is_6 = probs[0].p == 6.0;
  h->poly_ls = h->p_is_4 || h->p_is_6;
  h->ls_tx = L3_TX_WIDE;
  for (int b = 0; b < batch; ++b)
    if (probs[b].n < L3_TX_WIDE) h->ls_tx = L3_TX_NARROW;
  h->opt = *opt;
  h->mixed = opt->precision == PSD_MIXED;
  h->probs.assign(probs, probs + batch);
  auto fail = [&](const std::string& m) {
    h->err = m;
    return PSD_ERR_HIP;
  };
  // out of workspace: a HIP error with hipMalloc; with the static array a
  // problem too large for it, an argument error
  auto oom = [&]() {
    if (!h->arena) return fail("out of device memory");
    h->err = "the problem needs more workspace than the static scratch array of " +
             std::to_string(h->arena_cap >> 20) + " MiB";
    return PSD_ERR_ARG;
  };
  auto zero = [&](void* p, size_t bytes) {
    if (h->arena) {   // stream-ordered fill (the arena keeps the last call's contents)
      k_fill_zero<<<256, PSD_NT, 0, h->stream>>>((double*)p, (long long)(bytes / 8));
      return hipGetLastError();
    }
    return hipMemset(p, 0, bytes);
  };

  const size_t tds = h->mixed ? sizeof(float) : sizeof(double);
  h->hI.resize(batch);
  for (int b = 0; b < batch; ++b) {
    const psd_problem& P = probs[b];
    Inst& I = h->hI[b];
    std::memset(&I, 0, sizeof(Inst));
    I.dim = P.dim; I.n = P.n; I.nc = P.n / 2 + 1; I.order = P.order;
    I.ncell = (long long)P.n * P.n * (P.dim == 3 ? P.n : 1);
    {
      const long long rows = I.ncell / P.n;       // spectrum rows per field
      I.ncp32 = (P.n / 2 + 15) / 16 * 16;         // 16 FP32 complex = 128 bytes
      I.ncp64 = (P.n / 2 + 7) / 8 * 8;            // 8 FP64 complex = 128 bytes
      I.nyq32 = (long long)I.ncp32 * rows;
      I.nyq64 = (long long)I.ncp64 * rows;
      I.nspec32 = (I.nyq32 + rows + 15) / 16 * 16;
      I.nspec64 = (I.nyq64 + rows + 7) / 8 * 8;
      // buffer size per field in units of FP64 complex (16 bytes)
      I.nspec = std::max(I.nspec64, (I.nspec32 + 1) / 2);
    }
    I.h = P.L / P.n; I.inv_h = P.n / P.L; I.p = P.p; I.s = P.s;
    I.se2 = P.s * P.eps * P.eps; I.lam = P.lambda;
    I.inv_ntot = 1.0 / (double)I.ncell;
    I.tol = opt->tol;
    I.hd = std::pow(I.h, P.dim);
    I.max_iter = opt->max_iter;
    I.p_is_4 = P.p == 4.0; I.p_is_2 = P.p == 2.0; I.p_is_6 = P.p == 6.0;
    const size_t N = (size_t)I.ncell;
    const int nspec_fields = P.order == 6 ? 3 : 1;
    if (dalloc(h, &I.u[1], N * 8) || dalloc(h, &I.tmp, N * 8) ||
        dalloc(h, (char**)&I.d, N * tds) || dalloc(h, (char**)&I.r, N * tds) ||
        dalloc(h, (char**)&I.spec, (size_t)I.nspec * nspec_fields * 16) ||
        dalloc(h, (double**)&I.S, (size_t)P.n * 8) || dalloc(h, (char**)&I.tw32, (size_t)P.n * 8) ||
        dalloc(h, (char**)&I.tw64, (size_t)P.n * 16))
      return oom();
    if (P.order == 6) {
      if (dalloc(h, &I.w[0], N * 8) || dalloc(h, &I.w[1], N * 8) || dalloc(h, (char**)&I.e1, N * tds) ||
          dalloc(h, (char**)&I.e2, N * tds) || dalloc(h, (char**)&I.r1, N * tds))
        return oom();
    }
    if (zero(I.spec, (size_t)I.nspec * nspec_fields * 16) != hipSuccess)
      return fail("clearing the spectrum buffer failed");
    // symbol table of -Delta_h along one axis and twiddles (host, long double)
    std::vector<double> S(P.n);
    std::vector<float> t32(2 * (size_t)P.n);
    std::vector<double> t64(2 * (size_t)P.n);
    const long double pi = 3.141592653589793238462643383279502884L;
    for (int k = 0; k < P.n; ++k) {
      const long double sn = sinl(pi * k / P.n);
      S[k] = (double)(4.0L / ((long double)I.h * I.h) * sn * sn);
      const long double ang = -2.0L * pi * k / P.n;
      t64[2 * k] = (double)cosl(ang); t64[2 * k + 1] = (double)sinl(ang);
      t32[2 * k] = (float)t64[2 * k]; t32[2 * k + 1] = (float)t64[2 * k + 1];
    }
    if (hipMemcpy((void*)I.S, S.data(), S.size() * 8, hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy((void*)I.tw32, t32.data(), t32.size() * 4, hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy((void*)I.tw64, t64.data(), t64.size() * 8, hipMemcpyHostToDevice) != hipSuccess)
      return fail("copy of tables failed");
    if (opt->history && opt->max_iter > 0) {
      if (dalloc(h, &I.hist, (size_t)opt->max_iter * 4 * 8)) return oom();
      I.hist_cap = opt->max_iter;
    }
  }
  // task tables: capacities from the finest z-chunk, every line-search tile
  // width and the row layout with the most blocks (fewest lines per block)
  // that any tuning may pick
  std::vector<int> nsp_aux;
  std::vector<int> cap_res(batch, 0), cap_ls(batch, 0), cap_c2r(batch, 0);
  const int ls_tx0 = h->ls_tx;
  h->dT_cap = 0;
  h->row_sel = 0;
  for (int tx : {L3_TX_NARROW, ls_tx0}) {
    h->ls_tx = tx;
    h->tune_zc_res = h->tune_zc_ls = T3Z_MIN;
    build_all_tasks(h, nsp_aux);
    h->dT_cap = std::max(h->dT_cap, h->hT.size());
    for (int b = 0; b < batch; ++b) {
      cap_res[b] = std::max(cap_res[b], h->hI[b].nblk_res);
      cap_ls[b] = std::max(cap_ls[b], h->hI[b].nblk_ls);
      cap_c2r[b] = std::max(cap_c2r[b], h->hI[b].nblk_c2r);
    }
  }
  h->row_sel = 1;
  h->ls_tx = ls_tx0;
  h->tune_zc_res = T3Z_RES;
  h->tune_zc_ls = T3Z_LS;
  h->tune_xcd_res = h->tune_xcd_ls = false;
  build_all_tasks(h, nsp_aux);
  // partial arrays and states
  if (dalloc(h, &h->dState, sizeof(SolveState) * batch) || dalloc(h, &h->dAuxState, sizeof(SolveState) * batch))
    return oom();
  for (int b = 0; b < batch; ++b) {
    Inst& I = h->hI[b];
    const int nsp_max = std::max(I.nblk_sp, nsp_aux[b]);
    // adjoint vector kernels: a block per 2048 cells, 64 .. 1024 blocks
    I.nblk_vec = (int)std::min<long long>(1024, std::max<long long>(64, I.ncell / 2048));
    const int nres = std::max(cap_res[b], I.nblk_vec);
    if (dalloc(h, &I.part_res, (size_t)nres * 2 * 8) || dalloc(h, &I.part_ls, (size_t)cap_ls[b] * 8 * 8) ||
        dalloc(h, &I.part_sp, (size_t)nsp_max * 2 * 8) || dalloc(h, &I.part_c2r, (size_t)cap_c2r[b] * 3 * 8))
      return oom();
    I.st = h->dState + b;
  }
  if (dalloc(h, &h->dI, sizeof(Inst) * batch) || dalloc(h, &h->dT, sizeof(Task2) * h->dT_cap) ||
      dalloc(h, &h->dAuxPart, sizeof(double) * 5 * 1024))
    return oom();
  if (h->arena) {
    // host staging provided with the arena (no pinned allocation)
    h->hState = h->arena_hstate;
    h->hPart = h->arena_hpart;
  } else if (hipHostMalloc((void**)&h->hState, sizeof(SolveState) * batch, hipHostMallocDefault) != hipSuccess ||
             hipHostMalloc((void**)&h->hPart, sizeof(double) * 5 * 1024, hipHostMallocDefault) != hipSuccess) {
    return fail("pinned allocation failed");
  }
  std::memset(h->hState, 0, sizeof(SolveState) * batch);
  if (hipMemcpy(h->dT, h->hT.data(), sizeof(Task2) * h->hT.size(), hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(h->dI, h->hI.data(), sizeof(Inst) * batch, hipMemcpyHostToDevice) != hipSuccess ||
      zero(h->dState, sizeof(SolveState) * batch) != hipSuccess)
    return fail("upload of tables failed");
  return PSD_OK;
}

extern "C" psd_status psd_create(const psd_problem* probs, int batch, const psd_options* opt,
                                 void* hip_stream, psd_handle** out) {
  g_create_error.clear();
  if (!out) return set_err(nullptr, PSD_ERR_ARG, "out is NULL");
  *out = nullptr;
  std::string msg;
  psd_status cst = check_create_args(probs, batch, opt, msg);
  if (cst != PSD_OK) return set_err(nullptr, cst, msg);
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || ndev <= 0)
    return set_err(nullptr, PSD_ERR_HIP, "no HIP device");

  psd_handle* h = new psd_handle();
  (void)hipGetDevice(&h->device);
  if (hip_stream) h->stream = (hipStream_t)hip_stream;
  else {
    if (hipStreamCreate(&h->stream) != hipSuccess) { delete h; return set_err(nullptr, PSD_ERR_HIP, "stream"); }
    h->own_stream = true;
  }
  psd_status st = setup_handle(h, probs, batch, opt);
  if (st != PSD_OK) {
    std::string m = h->err;
    psd_destroy(h);
    return set_err(nullptr, st, m);
  }
  if (opt->autotune) {
    st = h->mixed ? autotune_impl<float, float>(h) : autotune_impl<double, double>(h);
    if (st != PSD_OK) {
      std::string m = "autotune: " + h->err;
      psd_destroy(h);
      return set_err(nullptr, st, m);
    }
  }
  *out = h;
  return PSD_OK;
}

extern "C" psd_status psd_tuning(const psd_handle* h, int* out6) {
  if (!h || !out6) return PSD_ERR_ARG;
  out6[0] = h->tune_zc_res; out6[1] = h->tune_zc_ls;
  out6[2] = h->tune_xcd_res ? 1 : 0; out6[3] = h->tune_xcd_ls ? 1 : 0;
  out6[4] = h->ls_tx;
  out6[5] = h->row_sel;
  return PSD_OK;
}

template <typename T, typename TD, typename TR>
static psd_status solve_impl(psd_handle* h, const double* const* f, const double* const* g, double* const* u,
                             double* const* w, psd_stats* stats) {
  const int B = h->batch;
  std::vector<int> pre_status(B, 0);
  for (int k = 0; k < PSD_NPASS; ++k) { h->pass_ms[k] = 0.0; h->pass_n[k] = 0; }
  if (!h->gexec) { h->prof.clear(); h->ev_used = 0; }
  // bind user buffers
  for (int b = 0; b < B; ++b) {
    Inst& I = h->hI[b];
    I.u[0] = u[b];
    I.f = f[b];
    I.g = (h->order == 6) ? g[b] : nullptr;
  }
  psd_status st = upload_inst(h);
  if (st != PSD_OK) return st;
  k_reset_state<<<(B + 63) / 64, 64, 0, h->stream>>>(h->dI, B);
  HIPCHK(hipGetLastError());
  if (h->order == 6) {
    // mean(u0) must equal mean(g); w0 = T_h(g - u0) + s lam gbar - fbar (Sec. 4)
    for (int b = 0; b < B; ++b) {
      Inst& I = h->hI[b];
      double su[3], sg[3];
      st = aux_sums(h, I.u[0], I.f, I.ncell, su);
      if (st != PSD_OK) return st;
      st = aux_sums(h, I.g, nullptr, I.ncell, sg);
      if (st != PSD_OK) return st;
      const double ubar = su[0] / I.ncell, fbar = su[1] / I.ncell, gbar = sg[0] / I.ncell;
      if (std::fabs(ubar - gbar) > 1e-12 * (1.0 + std::fabs(gbar))) pre_status[b] = PSD_ERR_MEAN;
      k_axpby<<<1024, PSD_NT, 0, h->stream>>>(I.tmp, I.g, I.u[0], 1.0, -1.0, 0.0, I.ncell);
    }
    // one auxiliary FP64 Poisson solve per instance (all instances at once)
    st = aux_poisson(h, 0, nullptr);
    if (st != PSD_OK) return st;
    for (int b = 0; b < B; ++b) {
      Inst& I = h->hI[b];
      double sf[3], sg[3];
      st = aux_sums(h, I.f, nullptr, I.ncell, sf);
      if (st != PSD_OK) return st;
      st = aux_sums(h, I.g, nullptr, I.ncell, sg);
      if (st != PSD_OK) return st;
      const double shift = I.s * I.lam * sg[0] / I.ncell - sf[0] / I.ncell;
      k_axpby<<<1024, PSD_NT, 0, h->stream>>>(I.w[0], I.tmp, nullptr, 1.0, 0.0, shift, I.ncell);
    }
  }
  for (int b = 0; b < B; ++b)
    if (pre_status[b]) k_set_status<<<1, 64, 0, h->stream>>>(h->dI, b, pre_status[b]);
  // initial residual (no update); graph-mode solves read its states with
  // the first queued replays in flight
  run_residual<TD, TR>(h, false);
  HIPCHK(hipGetLastError());
  const bool graph_mode = h->opt.graph_chunk > 0 && h->opt.metric != PSD_METRIC_VARIABLE;
  if (!graph_mode) {
    st = read_states(h);
    if (st != PSD_OK) return st;
  }
  if (graph_mode || !all_done(h)) {
    st = solve_loop<T, TD, TR>(h);
    if (st != PSD_OK) return st;
  }
  st = read_states(h);
  if (st != PSD_OK) return st;
  // move the final iterate (and w) to the caller's buffers
  psd_status worst = PSD_OK;
  for (int b = 0; b < B; ++b) {
    Inst& I = h->hI[b];
    const SolveState& S = h->hState[b];
    const int cur = S.iter & 1;
    if (cur == 1) HIPCHK(hipMemcpyAsync(u[b], I.u[1], I.ncell * 8, hipMemcpyDeviceToDevice, h->stream));
    if (h->order == 6 && w && w[b])
      HIPCHK(hipMemcpyAsync(w[b], I.w[cur], I.ncell * 8, hipMemcpyDeviceToDevice, h->stream));
    int status = pre_status[b] ? pre_status[b] : S.status;
    if (stats) {
      stats[b].iters = S.iter;
      stats[b].res_inf = S.rinf;
      stats[b].res_l2 = S.rl2;
      stats[b].status = status;
      stats[b].energy = NAN;
      stats[b].ls_truncated = S.ls_trunc;
    }
    if (status < 0 && (worst >= 0 || status < worst)) worst = (psd_status)status;
    else if (status > 0 && worst == PSD_OK) worst = (psd_status)status;
  }
  HIPCHK(hipStreamSynchronize(h->stream));
  // restore instance table pointers (u[0] = caller buffer is per call)
  if (stats && h->opt.history) {
    for (int b = 0; b < B; ++b) {
      double E = 0.0;
      psd_status es = psd_energy(h, b, f[b], h->order == 6 ? g[b] : nullptr, u[b], &E);
      if (es == PSD_OK) stats[b].energy = E;
    }
  }
  return worst;
}

extern "C" psd_status psd_solve(psd_handle* h, const double* const* f, const double* const* g,
                                double* const* u, double* const* w, psd_stats* stats) {
  if (!h) return PSD_ERR_ARG;
  if (!f || !u) return set_err(h, PSD_ERR_ARG, "f and u must be given");
  for (int b = 0; b < h->batch; ++b) {
    if (!f[b] || !u[b]) return set_err(h, PSD_ERR_ARG, "NULL f[b] or u[b]");
    if (h->order == 6 && (!g || !g[b])) return set_err(h, PSD_ERR_ARG, "order 6 needs g");
  }
  HIPCHK(hipSetDevice(h->device));
  if (h->mixed) return solve_impl<float, float, float>(h, f, g, u, w, stats);
  return solve_impl<double, double, double>(h, f, g, u, w, stats);
}

// ---------------------------------------------------------------------------
// Solve without allocating: every device buffer of the solve (iterate copy,
// search direction, residual copy, spectra, tables, partial sums, solver
// state, task lists) is carved from one static device array per GPU, and the
// host staging of the solver state lives in static host memory.
// ---------------------------------------------------------------------------
#define PSD_NOALLOC_BYTES ((size_t)64 << 20)
static __device__ __align__(256) double scratch[PSD_NOALLOC_BYTES / sizeof(double)];

namespace {
constexpr int PSD_NOALLOC_MAX_DEVICES = 64;
struct NoallocDevice {
  std::mutex mu;           // calls on one GPU run one after the other
  char* ptr = nullptr;     // device address of `scratch` on this GPU
  SolveState hstate[1];
  double hpart[5 * 1024];
};
NoallocDevice g_noalloc[PSD_NOALLOC_MAX_DEVICES];
}  // namespace

extern "C" psd_status psd_solve_noalloc(const psd_problem* prob, const psd_options* opt, void* hip_stream,
                                        const double* f, const double* g, double* u, double* w,
                                        psd_stats* stats) {
  g_create_error.clear();
  std::string msg;
  psd_status st = check_create_args(prob, 1, opt, msg);
  if (st != PSD_OK) return set_err(nullptr, st, msg);
  if (opt->graph_chunk != 0 || opt->profile || opt->autotune)
    return set_err(nullptr, PSD_ERR_ARG, "psd_solve_noalloc runs the host-driven loop: graph_chunk, "
                                         "profile and autotune must be 0");
  if (!f || !u || (prob->order == 6 && !g)) return set_err(nullptr, PSD_ERR_ARG, "NULL f, u or (order 6) g");
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= PSD_NOALLOC_MAX_DEVICES)
    return set_err(nullptr, PSD_ERR_HIP, "no HIP device");
  NoallocDevice& D = g_noalloc[dev];
  std::lock_guard<std::mutex> lock(D.mu);
  if (!D.ptr) {
    // the array's name is a host-side stand-in: its device address on this GPU
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p)
      return set_err(nullptr, PSD_ERR_HIP, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
    D.ptr = (char*)p;
  }
  psd_handle H;
  psd_handle* h = &H;
  h->device = dev;
  h->stream = (hipStream_t)hip_stream;
  h->arena = D.ptr;
  h->arena_cap = PSD_NOALLOC_BYTES;
  h->arena_hstate = D.hstate;
  h->arena_hpart = D.hpart;
  st = setup_handle(h, prob, 1, opt);
  if (st != PSD_OK) return set_err(nullptr, st, h->err);
  const double* const fa[1] = {f};
  const double* const ga[1] = {g};
  double* const ua[1] = {u};
  double* const wa[1] = {w};
  st = h->mixed ? solve_impl<float, float, float>(h, fa, ga, ua, wa, stats)
                : solve_impl<double, double, double>(h, fa, ga, ua, wa, stats);
  if (st < 0) set_err(nullptr, st, h->err.empty() ? std::string("solve failed") : h->err);
  (void)hipStreamSynchronize(h->stream);
  return st;
}

// ---------------------------------------------------------------------------
// Convex-splitting time stepping: one warm-started PSD solve per time level
// (Sec. 6.1 thin film, Sec. 6.2 SPFC).  The right-hand sides are formed on
// the device from the current level; the solve is psd_solve's.
// ---------------------------------------------------------------------------
template <typename T, typename TD, typename TR>
static psd_status timestep_impl(psd_handle* h, int scheme, double gamma1, double* const* u, double* const* w,
                                int nsteps, psd_step_stats* stats, int* step_iters) {
  const int B = h->batch;
  if (h->ts_f.empty()) {
    h->ts_f.assign(B, nullptr);
    h->ts_g.assign(B, nullptr);
    for (int b = 0; b < B; ++b) {
      const size_t bytes = (size_t)h->hI[b].ncell * 8;
      if (dalloc(h, &h->ts_f[b], bytes) || dalloc(h, &h->ts_g[b], bytes)) {
        h->ts_f.clear();
        h->ts_g.clear();
        return set_err(h, PSD_ERR_HIP, "out of device memory");
      }
    }
  }
  for (int b = 0; b < B; ++b) {
    stats[b].steps = 0; stats[b].psd_iters = 0; stats[b].max_iters = 0;
    stats[b].res_inf = 0.0; stats[b].status = PSD_OK;
  }
  std::vector<psd_stats> st1(B);
  const double* const* fa = h->ts_f.data();
  const double* const* ga = scheme == PSD_SCHEME_SPFC ? (const double* const*)h->ts_g.data() : nullptr;
  psd_status worst = PSD_OK;
  for (int step = 0; step < nsteps; ++step) {
    for (int b = 0; b < B; ++b)
      k_ts_rhs<<<1024, PSD_NT, 0, h->stream>>>(h->dI, b, scheme, gamma1, u[b], h->ts_f[b], h->ts_g[b]);
    HIPCHK(hipGetLastError());
    psd_status st = solve_impl<T, TD, TR>(h, fa, ga, u, w, st1.data());
    for (int b = 0; b < B; ++b) {
      psd_step_stats& S = stats[b];
      if (st1[b].status >= 0) S.steps += 1;
      S.psd_iters += st1[b].iters;
      S.max_iters = std::max(S.max_iters, st1[b].iters);
      S.res_inf = st1[b].res_inf;
      if (st1[b].status < 0 || (st1[b].status > 0 && S.status == PSD_OK)) S.status = st1[b].status;
      if (step_iters) step_iters[(size_t)step * B + b] = st1[b].iters;
    }
    if (st < 0) return st;
    if (st > 0) worst = st;
  }
  return worst;
}

extern "C" psd_status psd_timestep(psd_handle* h, int scheme, double gamma1, double* const* u, double* const* w,
                                   int nsteps, psd_step_stats* stats, int* step_iters) {
  if (!h) return PSD_ERR_ARG;
  if (!u || !stats || nsteps < 0) return set_err(h, PSD_ERR_ARG, "u and stats must be given, nsteps >= 0");
  for (int b = 0; b < h->batch; ++b)
    if (!u[b]) return set_err(h, PSD_ERR_ARG, "NULL u[b]");
  if (scheme == PSD_SCHEME_THINFILM) {
    if (h->order != 4) return set_err(h, PSD_ERR_ARG, "the thin-film scheme needs an order-4 problem");
  } else if (scheme == PSD_SCHEME_SPFC) {
    if (h->order != 6) return set_err(h, PSD_ERR_ARG, "the SPFC scheme needs an order-6 problem");
    if (!(gamma1 >= 0.0) || !std::isfinite(gamma1)) return set_err(h, PSD_ERR_RANGE, "gamma1 must be >= 0");
  } else {
    return set_err(h, PSD_ERR_ARG, "unknown scheme");
  }
  HIPCHK(hipSetDevice(h->device));
  if (h->mixed) return timestep_impl<float, float, float>(h, scheme, gamma1, u, w, nsteps, stats, step_iters);
  return timestep_impl<double, double, double>(h, scheme, gamma1, u, w, nsteps, stats, step_iters);
}

// Auxiliary single-instance evaluations (residual, energy, Poisson solves,
// adjoint) run on a separate state array: the state of the last solve
// (iteration count, residual norms, history length) survives them.  Every
// instance but `inst` (all when inst < 0) is marked finished, so their
// blocks return at once.
static psd_status aux_enter(psd_handle* h, int inst) {
  for (int b = 0; b < h->batch; ++b) h->hI[b].st = h->dAuxState + b;
  psd_status st = upload_inst(h);
  if (st != PSD_OK) return st;
  k_reset_state<<<(h->batch + 63) / 64, 64, 0, h->stream>>>(h->dI, h->batch);
  if (inst >= 0) k_mark_done<<<(h->batch + 63) / 64, 64, 0, h->stream>>>(h->dI, h->batch, inst);
  HIPCHK(hipGetLastError());
  return PSD_OK;
}

static psd_status aux_leave(psd_handle* h) {
  for (int b = 0; b < h->batch; ++b) h->hI[b].st = h->dState + b;
  return upload_inst(h);
}

// Evaluate the residual kernel once for instance `inst` at caller buffers,
// writing FP64 r (and r1 for order 6) without an update.
static psd_status aux_residual(psd_handle* h, int inst, const double* f, const double* g, const double* u,
                               const double* wv, double* r2out, double* r1out, double* res_inf) {
  Inst saved = h->hI[inst];
  Inst& I = h->hI[inst];
  I.u[0] = const_cast<double*>(u);
  I.f = f;
  I.g = g;
  I.r = r2out;
  if (h->order == 6) { I.w[0] = const_cast<double*>(wv); I.r1 = r1out; }
  psd_status st = aux_enter(h, inst);   // other instances marked done
  if (st == PSD_OK) {
    run_residual<double, double>(h, false);
    st = hipGetLastError() == hipSuccess ? read_states(h) : PSD_ERR_HIP;
    if (st == PSD_OK && res_inf) *res_inf = h->hState[inst].rinf;
  }
  saved.st = h->dState + inst;
  h->hI[inst] = saved;
  psd_status st2 = aux_leave(h);
  HIPCHK(hipStreamSynchronize(h->stream));
  return st != PSD_OK ? st : st2;
}

extern "C" psd_status psd_residual(psd_handle* h, int inst, const double* f, const double* g, const double* u,
                                   double* r, double* res_inf) {
  if (!h) return PSD_ERR_ARG;
  if (inst < 0 || inst >= h->batch || !f || !u || (h->order == 6 && !g))
    return set_err(h, PSD_ERR_ARG, "bad arguments");
  HIPCHK(hipSetDevice(h->device));
  Inst& I = h->hI[inst];
  if (h->order == 4) {
    double* rr = r ? r : I.tmp;
    return aux_residual(h, inst, f, g, u, nullptr, rr, nullptr, res_inf);
  }
  // order 6: w = T_h(g - u); r2 = f - (s lam u - s div + s eps^2 Delta^2 u - w); rho = r2 - mean(r2)
  k_axpby<<<1024, PSD_NT, 0, h->stream>>>(I.tmp, g, u, 1.0, -1.0, 0.0, I.ncell);
  // the auxiliary transform runs on instance inst only
  psd_status st = aux_enter(h, inst);
  if (st == PSD_OK) st = aux_poisson(h, inst, nullptr);
  psd_status st2 = aux_leave(h);
  if (st != PSD_OK) return st;
  if (st2 != PSD_OK) return st2;
  double* rr = r ? r : (double*)I.d;  // FP64 scratch of ncell doubles needed
  double* wtmp = I.u[1];
  HIPCHK(hipMemcpyAsync(wtmp, I.tmp, I.ncell * 8, hipMemcpyDeviceToDevice, h->stream));
  if (!r) {
    // no caller buffer: use tmp for r2 (w copied to u[1] above)
    rr = I.tmp;
  }
  double* r1 = I.w[1];
  st = aux_residual(h, inst, f, g, u, wtmp, rr, r1, nullptr);
  if (st != PSD_OK) return st;
  double sm[3];
  st = aux_sums(h, rr, nullptr, I.ncell, sm);
  if (st != PSD_OK) return st;
  k_axpby<<<1024, PSD_NT, 0, h->stream>>>(rr, rr, nullptr, 1.0, 0.0, -sm[0] / I.ncell, I.ncell);
  if (res_inf) {
    // max-norm on the host copy (auxiliary path, not performance relevant)
    std::vector<double> host((size_t)I.ncell);
    HIPCHK(hipMemcpyAsync(host.data(), rr, I.ncell * 8, hipMemcpyDeviceToHost, h->stream));
    HIPCHK(hipStreamSynchronize(h->stream));
    double m = 0.0;
    for (double v : host) m = std::max(m, std::fabs(v));
    *res_inf = m;
  }
  HIPCHK(hipStreamSynchronize(h->stream));
  return PSD_OK;
}

extern "C" psd_status psd_residual_mixed(psd_handle* h, int inst, const double* f, const double* g,
                                         const double* u, const double* w, double* r1, double* r2,
                                         double* res_inf) {
  if (!h) return PSD_ERR_ARG;
  if (h->order != 6) return set_err(h, PSD_ERR_ARG, "psd_residual_mixed needs order 6");
  if (inst < 0 || inst >= h->batch || !f || !g || !u || !w) return set_err(h, PSD_ERR_ARG, "bad arguments");
  HIPCHK(hipSetDevice(h->device));
  Inst& I = h->hI[inst];
  return aux_residual(h, inst, f, g, u, w, r2 ? r2 : I.tmp, r1 ? r1 : I.u[1], res_inf);
}

extern "C" psd_status psd_energy(psd_handle* h, int inst, const double* f, const double* g, const double* u,
                                 double* E) {
  if (!h) return PSD_ERR_ARG;
  if (inst < 0 || inst >= h->batch || !f || !u || !E || (h->order == 6 && !g))
    return set_err(h, PSD_ERR_ARG, "bad arguments");
  HIPCHK(hipSetDevice(h->device));
  Inst& I = h->hI[inst];
  const int nblk = 1024;
  k_energy_parts<<<nblk, PSD_NT, 0, h->stream>>>(h->dI, inst, u, f, h->dAuxPart);
  HIPCHK(hipGetLastError());
  HIPCHK(hipMemcpyAsync(h->hPart, h->dAuxPart, sizeof(double) * 5 * nblk, hipMemcpyDeviceToHost, h->stream));
  HIPCHK(hipStreamSynchronize(h->stream));
  double a[5] = {0, 0, 0, 0, 0};
  for (int k = 0; k < nblk; ++k)
    for (int q = 0; q < 5; ++q) a[q] += h->hPart[5 * k + q];
  const double s = I.s, se2 = I.se2, p = I.p;
  if (h->order == 4) {
    *E = I.hd * (0.5 * a[0] + s / p * a[1] + 0.5 * se2 * a[2]);
    return PSD_OK;
  }
  // order 6 at nu = u - gbar: 1/2 (z, T z) + lam s/2 ||u||^2 - (nu, f) + s/p sum|G|^p + s eps^2/2 sum (Delta u)^2
  double sg[3], sf[3];
  psd_status st = aux_sums(h, g, nullptr, I.ncell, sg);
  if (st != PSD_OK) return st;
  st = aux_sums(h, f, nullptr, I.ncell, sf);
  if (st != PSD_OK) return st;
  const double gbar = sg[0] / I.ncell;
  k_axpby<<<1024, PSD_NT, 0, h->stream>>>(I.tmp, u, g, 1.0, -1.0, 0.0, I.ncell);
  double zTz = 0.0;
  st = aux_enter(h, inst);
  if (st == PSD_OK) st = aux_poisson(h, inst, &zTz);
  psd_status st2 = aux_leave(h);
  if (st != PSD_OK) return st;
  if (st2 != PSD_OK) return st2;
  *E = I.hd * (0.5 * zTz + 0.5 * I.lam * s * a[3] - (a[4] - gbar * sf[0]) + s / p * a[1] + 0.5 * se2 * a[2]);
  return PSD_OK;
}

extern "C" psd_status psd_grad(psd_handle* h, int inst, const double* f, const double* g, const double* u,
                               double* grad) {
  if (!h) return PSD_ERR_ARG;
  if (inst < 0 || inst >= h->batch || !f || !u || !grad || (h->order == 6 && !g))
    return set_err(h, PSD_ERR_ARG, "bad arguments");
  psd_status st = psd_residual(h, inst, f, g, u, grad, nullptr);
  if (st != PSD_OK) return st;
  Inst& I = h->hI[inst];
  k_axpby<<<1024, PSD_NT, 0, h->stream>>>(grad, grad, nullptr, -1.0, 0.0, 0.0, I.ncell);
  HIPCHK(hipGetLastError());
  HIPCHK(hipStreamSynchronize(h->stream));
  return PSD_OK;
}

extern "C" psd_status psd_history(psd_handle* h, int inst, double* out, int cap, int* count) {
  if (!h) return PSD_ERR_ARG;
  if (inst < 0 || inst >= h->batch || !out || !count) return set_err(h, PSD_ERR_ARG, "bad arguments");
  const Inst& I = h->hI[inst];
  if (!I.hist) { *count = 0; return set_err(h, PSD_ERR_ARG, "history was not enabled"); }
  HIPCHK(hipSetDevice(h->device));
  HIPCHK(hipStreamSynchronize(h->stream));
  SolveState S;
  HIPCHK(hipMemcpy(&S, I.st, sizeof(SolveState), hipMemcpyDeviceToHost));
  const int k = std::min(std::min(S.iter, I.hist_cap), cap);
  if (k > 0) HIPCHK(hipMemcpy(out, I.hist, sizeof(double) * 4 * k, hipMemcpyDeviceToHost));
  *count = k;
  return PSD_OK;
}

// Conjugate-gradient buffers (residual, direction, operator times direction),
// allocated once per handle; shared by the adjoint and the variable metric.
static psd_status ensure_cg_buffers(psd_handle* h) {
  if (h->adj_alloc) return PSD_OK;
  for (int b = 0; b < h->batch; ++b) {
    Inst& I = h->hI[b];
    if (dalloc(h, &I.adj_r, I.ncell * 8) || dalloc(h, &I.adj_p, I.ncell * 8) || dalloc(h, &I.adj_Hp, I.ncell * 8))
      return set_err(h, PSD_ERR_HIP, "out of device memory");
  }
  h->adj_alloc = true;
  return PSD_OK;
}

// Flexible conjugate gradients on  A lam = g  for every instance, A the Hessian
// of E_h at adj_us (second variation, Sec. 5.3) or, with adj_frozen, the
// variable metric L_k; preconditioned by L_h^{-1} (the FFT passes).  The
// instance table must point at the auxiliary states (reset, finished
// instances marked done), adj_g/adj_lam/adj_us at the fields, max_iter at the
// iteration cap.  Stops at ||res||_2^2 <= rtol2 ||g||_2^2 or the cap; the host
// reads the states after every iteration.
template <typename T, typename TD, typename TR>
static psd_status cg_solve(psd_handle* h, double rtol2, int max_iter) {
  const int B = h->batch;
  hipStream_t s = h->stream;
  int nmax = 1;
  for (int b = 0; b < B; ++b) nmax = std::max(nmax, h->hI[b].nblk_vec);
  auto vec = [&](int op) { k_cg_vec<TD, TR><<<B * nmax, PSD_NT, 0, s>>>(h->dI, nmax, op); };
  auto fin = [&](int mode) {
    // vector partials: nblk_vec per instance (read from the instance table)
    k_cg_fin<<<B, PSD_NT, 0, s>>>(h->dI, mode, -1, rtol2);
  };
  vec(0);
  fin(0);
  run_fft<T, TR, TD>(h, h->fft_solver, OP_PRECOND4, true);
  fin(1);
  vec(3);
  const Task2* tt = h->dT + h->res.off;
  for (int it = 0; it < max_iter; ++it) {
    if (h->dim == 2) k_hess2d<TD, TR><<<h->res.cnt, PSD_NT, (R2_LDS + 16) * sizeof(double), s>>>(h->dI, tt);
    else k_hess3d<TR, R3_TX><<<h->res.cnt, PSD_NT, (R3Shape<R3_TX>::HLDS + 16) * sizeof(double), s>>>(h->dI, tt);
    fin(2);
    vec(1);
    fin(3);
    HIPCHK(hipGetLastError());
    psd_status st = read_states(h);
    if (st != PSD_OK) return st;
    if (all_done(h)) break;
    run_fft<T, TR, TD>(h, h->fft_solver, OP_PRECOND4, true);
    vec(2);
    fin(4);
    vec(4);
  }
  return read_states(h);
}

template <typename T, typename TD, typename TR>
static psd_status adjoint_impl(psd_handle* h, const double* const* u_star, const double* const* dJdu,
                               double* const* dJdf, double* dJds, double* dJdeps, double rtol, int max_iter,
                               int* cg_iters) {
  const int B = h->batch;
  hipStream_t s = h->stream;
  psd_status st = ensure_cg_buffers(h);
  if (st != PSD_OK) return st;
  std::vector<Inst> saved = h->hI;
  for (int b = 0; b < B; ++b) {
    Inst& I = h->hI[b];
    I.adj_us = u_star[b];
    I.adj_g = dJdu[b];
    I.adj_lam = dJdf[b];
    I.max_iter = max_iter;
    I.adj_frozen = 0;
    I.st = h->dAuxState + b;   // the CG state; the last solve's state stays intact
  }
  st = upload_inst(h);
  if (st != PSD_OK) { h->hI = saved; (void)upload_inst(h); return st; }
  k_reset_state<<<(B + 63) / 64, 64, 0, s>>>(h->dI, B);
  st = cg_solve<T, TD, TR>(h, rtol * rtol, max_iter);
  if (st != PSD_OK) { h->hI = saved; (void)upload_inst(h); return st; }
  psd_status worst = PSD_OK;
  // sensitivities to s and eps (one pass per instance)
  const int nblk = 1024;
  for (int b = 0; b < B; ++b) {
    const Inst& I = h->hI[b];
    const SolveState& S = h->hState[b];
    if (cg_iters) cg_iters[b] = S.iter;
    if (S.status < 0) worst = (psd_status)S.status;
    else if (S.status > 0 && worst == PSD_OK) worst = PSD_NOT_CONVERGED;
    k_param_sens<<<nblk, PSD_NT, 0, s>>>(h->dI, b, h->dAuxPart);
    HIPCHK(hipGetLastError());
    HIPCHK(hipMemcpyAsync(h->hPart, h->dAuxPart, sizeof(double) * 3 * nblk, hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    double a0 = 0.0, a1 = 0.0;
    for (int k = 0; k < nblk; ++k) { a0 += h->hPart[3 * k]; a1 += h->hPart[3 * k + 1]; }
    // dN/ds = -plap(u*) + eps^2 Delta_h^2 u*,  dN/deps = 2 s eps Delta_h^2 u*
    const double eps = std::sqrt(I.se2 / I.s);
    if (dJds) dJds[b] = -a0;
    if (dJdeps) dJdeps[b] = -2.0 * I.s * eps * a1;
  }
  h->hI = saved;
  st = upload_inst(h);
  HIPCHK(hipStreamSynchronize(s));
  return st != PSD_OK ? st : worst;
}

// Variable-metric search direction (Remark in Sec. 3): d = L_k^{-1} r with
// L_k = I - s div_h(|grad_h u^k|^{p-2} grad_h .) + s eps^2 Delta_h^2 by the
// conjugate gradients above (operator flag adj_frozen), on the auxiliary
// states so the PSD state is untouched.  The FP64 residual goes to tmp, the
// solution to the iterate buffer the next update overwrites; at the end the
// solution becomes d and the spectral partial slots receive (r, d) for -q(0).
// hState must hold the PSD states (iteration parity of each instance).
template <typename T, typename TD, typename TR>
static psd_status vm_direction(psd_handle* h) {
  const int B = h->batch;
  hipStream_t s = h->stream;
  psd_status st = ensure_cg_buffers(h);
  if (st != PSD_OK) return st;
  std::vector<Inst> saved = h->hI;
  for (int b = 0; b < B; ++b) {
    Inst& I = h->hI[b];
    const int cur = h->hState[b].iter & 1;
    I.adj_us = I.u[cur];
    I.adj_g = I.tmp;
    I.adj_lam = I.u[cur ^ 1];
    I.max_iter = h->opt.inner_iters;
    I.adj_frozen = 1;
    I.st = h->dAuxState + b;
  }
  st = upload_inst(h);
  if (st != PSD_OK) { h->hI = saved; (void)upload_inst(h); return st; }
  k_reset_state<<<(B + 63) / 64, 64, 0, s>>>(h->dI, B);
  for (int b = 0; b < B; ++b) k_vm_start<TR><<<h->hI[b].nblk_vec, PSD_NT, 0, s>>>(h->dI, b, h->dState);
  HIPCHK(hipGetLastError());
  st = cg_solve<T, TD, TR>(h, h->opt.inner_rtol * h->opt.inner_rtol, h->opt.inner_iters);
  // back to the PSD states; the CG fields stay bound for the hand-over
  for (int b = 0; b < B; ++b) {
    Inst& I = h->hI[b];
    I.st = saved[b].st;
    I.max_iter = saved[b].max_iter;
    I.adj_frozen = 0;
  }
  psd_status st2 = upload_inst(h);
  if (st != PSD_OK) return st;
  if (st2 != PSD_OK) return st2;
  for (int b = 0; b < B; ++b) k_vm_finish<TD><<<h->hI[b].nblk_sp, PSD_NT, 0, s>>>(h->dI, b);
  HIPCHK(hipGetLastError());
  return PSD_OK;
}

// Adjoint of the converged sixth-order solve on the mean-zero space (Sec. 4,
// Sec. 5.4): H Lam = P0 G with H = s lam - s (linearised p-Laplacian) +
// s eps^2 Delta_h^2 + T_h, conjugate gradients preconditioned by the one-field
// sixth-order L_h^{-1}, in FP64 (T_h and L_h^{-1} on the auxiliary FP64
// transform of tmp), on the auxiliary states.
static psd_status adjoint6_impl(psd_handle* h, const double* const* u_star, const double* const* dJdu,
                                double* const* dJdf, double* const* dJdg, double* dJds, double* dJdeps,
                                double* dJdlam, double rtol, int max_iter, int* cg_iters) {
  const int B = h->batch;
  hipStream_t s = h->stream;
  psd_status st = ensure_cg_buffers(h);
  if (st != PSD_OK) return st;
  std::vector<Inst> saved = h->hI;
  for (int b = 0; b < B; ++b) {
    Inst& I = h->hI[b];
    I.adj_us = u_star[b];
    I.adj_g = dJdu[b];
    I.adj_lam = dJdf[b];
    I.max_iter = max_iter;
    I.adj_frozen = 0;
    I.st = h->dAuxState + b;
  }
  auto restore = [&]() { h->hI = saved; return upload_inst(h); };
  st = upload_inst(h);
  if (st != PSD_OK) { (void)restore(); return st; }
  k_reset_state<<<(B + 63) / 64, 64, 0, s>>>(h->dI, B);
  const double rtol2 = rtol * rtol;
  int nmax = 1;
  for (int b = 0; b < B; ++b) nmax = std::max(nmax, h->hI[b].nblk_vec);
  auto vec = [&](int op) { k_cg6_vec<<<B * nmax, PSD_NT, 0, s>>>(h->dI, nmax, op); };
  auto fin = [&](int mode) { k_cg6_fin<<<B, PSD_NT, 0, s>>>(h->dI, mode, rtol2); };
  auto aux_fft = [&](int op) { run_fft<double, double, double>(h, h->fft_aux, op, false); };
  const Task2* tt = h->dT + h->res.off;
  auto hess = [&]() {
    if (h->dim == 2) k_hess2d<double, double, 6><<<h->res.cnt, PSD_NT, (R2_LDS + 16) * sizeof(double), s>>>(h->dI, tt);
    else k_hess3d6<<<h->res.cnt, PSD_NT, (B6_LDS + 16) * sizeof(double), s>>>(h->dI, tt);
  };
  vec(0); fin(0);                 // mean of G
  vec(1); fin(1);                 // r = P0 G, threshold
  aux_fft(OP_PRECOND6S);          // z = L^-1 r in tmp
  vec(2); fin(2);                 // r.z
  vec(3);                         // p = z
  for (int it = 0; it < max_iter; ++it) {
    hess();                       // stencil part of H p
    vec(4);                       // tmp = p
    aux_fft(OP_POISSON);          // tmp = T_h p
    vec(5); fin(3);               // Hp += T_h p, alpha
    vec(6); fin(4);               // lam, r, stop test; tmp = r
    HIPCHK(hipGetLastError());
    st = read_states(h);
    if (st != PSD_OK) { (void)restore(); return st; }
    if (all_done(h)) break;
    aux_fft(OP_PRECOND6S);        // z = L^-1 r
    vec(7); fin(5);               // beta, r.z
    vec(8);                       // p = z + beta p
  }
  st = read_states(h);
  if (st != PSD_OK) { (void)restore(); return st; }
  psd_status worst = PSD_OK;
  const int nblk = 1024;
  for (int b = 0; b < B; ++b) {
    const Inst& I = h->hI[b];
    const SolveState& S = h->hState[b];
    if (cg_iters) cg_iters[b] = S.iter;
    if (S.status < 0) worst = (psd_status)S.status;
    else if (S.status > 0 && worst == PSD_OK) worst = PSD_NOT_CONVERGED;
    // dJ/dg = sum(G)/N + T_h Lam (tmp <- Lam, auxiliary Poisson solve of this instance)
    HIPCHK(hipMemcpyAsync(I.tmp, I.adj_lam, I.ncell * 8, hipMemcpyDeviceToDevice, s));
  }
  aux_fft(OP_POISSON);
  for (int b = 0; b < B; ++b) {
    const Inst& I = h->hI[b];
    const SolveState& S = h->hState[b];
    if (dJdg && dJdg[b])
      k_axpby<<<1024, PSD_NT, 0, s>>>(dJdg[b], I.tmp, nullptr, 1.0, 0.0, S.lo, I.ncell);   // S.lo = sum(G)/N
    k_param_sens<<<nblk, PSD_NT, 0, s>>>(h->dI, b, h->dAuxPart);
    HIPCHK(hipGetLastError());
    HIPCHK(hipMemcpyAsync(h->hPart, h->dAuxPart, sizeof(double) * 3 * nblk, hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    double a0 = 0.0, a1 = 0.0, a2 = 0.0;
    for (int k = 0; k < nblk; ++k) { a0 += h->hPart[3 * k]; a1 += h->hPart[3 * k + 1]; a2 += h->hPart[3 * k + 2]; }
    // dN/ds = lam u - plap(u) + eps^2 Delta_h^2 u, dN/deps = 2 s eps Delta_h^2 u, dN/dlam = s u
    const double eps = std::sqrt(I.se2 / I.s);
    if (dJds) dJds[b] = -(a0 + I.lam * a2);
    if (dJdeps) dJdeps[b] = -2.0 * I.s * eps * a1;
    if (dJdlam) dJdlam[b] = -I.s * a2;
  }
  st = restore();
  HIPCHK(hipStreamSynchronize(s));
  return st != PSD_OK ? st : worst;
}

extern "C" psd_status psd_adjoint6(psd_handle* h, const double* const* u_star, const double* const* dJdu,
                                   double* const* dJdf, double* const* dJdg, double* dJds, double* dJdeps,
                                   double* dJdlam, double rtol, int max_iter, int* cg_iters) {
  if (!h) return PSD_ERR_ARG;
  if (h->order != 6) return set_err(h, PSD_ERR_ARG, "psd_adjoint6 needs an order-6 problem");
  if (!u_star || !dJdu || !dJdf || max_iter <= 0 || !(rtol >= 0.0)) return set_err(h, PSD_ERR_ARG, "bad arguments");
  for (int b = 0; b < h->batch; ++b)
    if (!u_star[b] || !dJdu[b] || !dJdf[b]) return set_err(h, PSD_ERR_ARG, "NULL instance pointer");
  HIPCHK(hipSetDevice(h->device));
  return adjoint6_impl(h, u_star, dJdu, dJdf, dJdg, dJds, dJdeps, dJdlam, rtol, max_iter, cg_iters);
}

extern "C" psd_status psd_adjoint(psd_handle* h, const double* const* u_star, const double* const* dJdu,
                                  double* const* dJdf, double* dJds, double* dJdeps, double rtol, int max_iter,
                                  int* cg_iters) {
  if (!h) return PSD_ERR_ARG;
  if (h->order != 4) return set_err(h, PSD_ERR_ARG, "the adjoint is available for order 4");
  if (!u_star || !dJdu || !dJdf || max_iter <= 0 || !(rtol >= 0.0)) return set_err(h, PSD_ERR_ARG, "bad arguments");
  for (int b = 0; b < h->batch; ++b)
    if (!u_star[b] || !dJdu[b] || !dJdf[b]) return set_err(h, PSD_ERR_ARG, "NULL instance pointer");
  HIPCHK(hipSetDevice(h->device));
  if (h->mixed) return adjoint_impl<float, float, float>(h, u_star, dJdu, dJdf, dJds, dJdeps, rtol, max_iter, cg_iters);
  return adjoint_impl<double, double, double>(h, u_star, dJdu, dJdf, dJds, dJdeps, rtol, max_iter, cg_iters);
}

extern "C" psd_status psd_pass_times(psd_handle* h, double* ms, int* launches) {
  if (!h) return PSD_ERR_ARG;
  if (!ms || !launches) return set_err(h, PSD_ERR_ARG, "NULL output");
  for (int k = 0; k < PSD_NPASS; ++k) { ms[k] = h->pass_ms[k]; launches[k] = h->pass_n[k]; }
  return PSD_OK;
}

extern "C" psd_status psd_destroy(psd_handle* h) {
  if (!h) return PSD_ERR_ARG;
  (void)hipSetDevice(h->device);
  if (h->stream) (void)hipStreamSynchronize(h->stream);
  if (h->gexec) (void)hipGraphExecDestroy(h->gexec);
  if (h->graph) (void)hipGraphDestroy(h->graph);
  for (void* p : h->allocs) (void)hipFree(p);
  for (hipEvent_t e : h->ev_pool) (void)hipEventDestroy(e);
  if (h->hState) (void)hipHostFree(h->hState);
  if (h->hPart) (void)hipHostFree(h->hPart);
  for (int k = 0; k < 2; ++k) {
    if (h->hStateQ[k]) (void)hipHostFree(h->hStateQ[k]);
    if (h->ev_state[k]) (void)hipEventDestroy(h->ev_state[k]);
  }
  if (h->own_stream && h->stream) (void)hipStreamDestroy(h->stream);
  delete h;
  return PSD_OK;
}

extern "C" const char* psd_last_error(const psd_handle* h) {
  if (!h) return g_create_error.c_str();
  return h->err.c_str();
}
