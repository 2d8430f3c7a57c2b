// C ABI of the space-time GMRES-GMG solver: hierarchy setup, V-cycle with the
// patchwise Vanka smoother (Def:VankaOP, Algorithm 4.1), flexible GMRES
// (Sec. 4) and test entry points.  Host code orchestrating the kernels of
// kernels.hip on the handle's stream.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <complex>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <memory>
#include <mutex>
#include <new>
#include <stdexcept>
#include <string>
#include <thread>
#include <vector>

#include "host_setup.h"
#include "kernels.h"
#include "stgmg.h"

// Workspace of stgmg_solve_noalloc: one file-scope device array, so that the call allocates
// nothing.  Every GPU the library runs on holds its own copy (loaded with the code object) until
// the process ends.  Host code never passes `scratch` itself to a kernel (on the host the name
// is only a stand-in for the symbol): it uses the device address that hipGetSymbolAddress returns
// for the current device, kept per device in g_scratch.
static __device__ __align__(256) double scratch[STGMG_NOALLOC_SCRATCH_BYTES / sizeof(double)];

namespace {

thread_local std::string g_last_error;

constexpr int MAX_DEVICES = 64;
std::mutex g_scratch_mu;
double* g_scratch[MAX_DEVICES] = {};  // device address of `scratch` on each device, once looked up

struct ApiError : std::runtime_error {
  stgmg_status code;
  ApiError(stgmg_status c, const std::string& m) : std::runtime_error(m), code(c) {}
};

#define HIPCHK(expr)                                                                                  \
  do {                                                                                                \
    hipError_t e_ = (expr);                                                                           \
    if (e_ != hipSuccess) {                                                                           \
      throw ApiError(e_ == hipErrorOutOfMemory ? STGMG_ERR_OOM : STGMG_ERR_HIP,                       \
                     std::string(#expr) + ": " + hipGetErrorString(e_));                              \
    }                                                                                                 \
  } while (0)

// Owning device array, allocated and freed stream-ordered on the stream given
// at allocation (the owning handle's stream), so that releasing one problem's
// memory does not synchronise the device for the other problems.
template <class T>
struct DArr {
  T* p = nullptr;
  int64_t n = 0;
  hipStream_t s = nullptr;
  DArr() = default;
  DArr(const DArr&) = delete;
  DArr& operator=(const DArr&) = delete;
  DArr(DArr&& o) noexcept : p(o.p), n(o.n), s(o.s) {
    o.p = nullptr;
    o.n = 0;
  }
  DArr& operator=(DArr&& o) noexcept {
    if (this != &o) {
      release();
      p = o.p;
      n = o.n;
      s = o.s;
      o.p = nullptr;
      o.n = 0;
    }
    return *this;
  }
  ~DArr() { release(); }
  void release() {
    if (p) (void)hipFreeAsync(p, s);
    p = nullptr;
    n = 0;
  }
  void alloc(int64_t count, int64_t* counter, hipStream_t stream) {
    release();
    s = stream;
    if (count > 0) HIPCHK(hipMallocAsync(reinterpret_cast<void**>(&p), size_t(count) * sizeof(T), s));
    n = count;
    if (counter) *counter += count * int64_t(sizeof(T));
  }
  void upload(const std::vector<T>& h, hipStream_t st, int64_t* counter) {
    alloc(int64_t(h.size()), counter, st);
    if (!h.empty()) HIPCHK(hipMemcpyAsync(p, h.data(), h.size() * sizeof(T), hipMemcpyHostToDevice, st));
  }
};

struct DevCsr {
  int64_t nrows = 0, nnz = 0;
  int lanes = 16;
  DArr<int64_t> ptr;
  DArr<int32_t> col;
  DArr<double> val;
  void upload(const stgmg::Csr& c, hipStream_t st, int64_t* counter) {
    nrows = c.nrows;
    nnz = int64_t(c.col.size());
    ptr.upload(c.ptr, st, counter);
    col.upload(c.col, st, counter);
    val.upload(c.val, st, counter);
    const double avg = nrows ? double(nnz) / double(nrows) : 0.0;
    lanes = avg < 12 ? 4 : avg < 24 ? 8 : avg < 100 ? 16 : avg < 200 ? 32 : 64;
    if (const char* e = std::getenv("STGMG_CSR_LANES")) {  // tuning override: lanes per row for rows of > 24 entries
      const int v = std::atoi(e);
      if ((v == 4 || v == 8 || v == 16 || v == 32 || v == 64) && avg >= 24) lanes = v;
    }
  }
  void apply(hipStream_t st, int mode, const double* x, const double* b, double* y) const {
    stgmg::k_csr(st, mode, nrows, ptr.p, col.p, val.p, x, b, y, lanes);
  }
};

struct LevelDev {
  int N = 0;
  int64_t n = 0, ns = 0;
  DevCsr A;
  int64_t npatch = 0;
  int max_np = 0;
  DArr<int64_t> poff, ioff, tptr;
  DArr<int32_t> tpos;  // dof-major slot of each patch entry
  DArr<int32_t> pdof;
  DArr<int32_t> pnu;  // reduced solves: velocity dofs nU per patch (one time node)
  int max_nu = 0, max_nr = 0, max_npr = 0;
  bool sym = false;  // reduced solves with the Schur inverses as symmetric tiles
  int waves = 0;     // waves per patch of the tiled patch kernel on this level (0: by patch count)
  DArr<double> inv64, winv, y;
  DArr<float> inv32;
  DArr<__bf16> inv16;  // BF16 storage (symmetric tiles and the small reduced factors)
  DevCsr P, R;  // prolongation from level-1 and its transpose
  DevCsr MMs, KKs;  // spatial MM and KK: the level operator A = D^t (x) MM + M^t (x) KK
  // the velocity rows of the same operator by node pairs (rhoM_ij, A_ij, C^T), used by the
  // residual and operator kernel when the level has that structure (node_ok)
  bool node_ok = false;
  stgmg::NodeOpDev node{};
  DArr<int64_t> nptr, ncptr;
  DArr<int32_t> ncol, nccol;
  DArr<double> nm, na, nc;
  double alg_op_values = 0;  // values the operator kernel reads (node form: each stored once)
  int op_lanes = 16;
  double alg_inv_entries = 0;  // stored inverse values excluding padding
  DArr<double> b, d, r;
  std::vector<int64_t> poff_h, ioff_h;
  std::vector<int32_t> pdof_h, pnu_h;
};

}  // namespace

// The handle's own stream.  Declared as the first member of the handle so that it is
// destroyed last: every device array is freed stream-ordered on it before.
struct OwnStream {
  hipStream_t s = nullptr;
  ~OwnStream() {
    if (s) {
      (void)hipStreamSynchronize(s);
      (void)hipStreamDestroy(s);
    }
  }
};

struct stgmg_handle {
  OwnStream own;
  stgmg_params prm{};
  hipStream_t st = nullptr;      // == own.s (default priority, non-blocking)
  hipStream_t caller = nullptr;  // the caller's stream: each call waits for it first
  hipEvent_t enter_ev = nullptr;
  hipEvent_t vc_ev[2] = {nullptr, nullptr};  // around each V-cycle of a solve (stgmg_info.t_vcycle_ms)
  int dev = 0;  // the device current at setup (its static scratch serves stgmg_solve_noalloc)
  // V-cycle graph: z = B r with r read from gin and z written to gout
  bool use_graph = false;
  hipGraphExec_t graph_exec = nullptr;
  hipGraph_t graph = nullptr;
  int L = 0;  // finest level index
  std::vector<LevelDev> lv;
  int64_t bytes = 0;
  // coarse solve
  int n0 = 0;
  DArr<double> coarse_inv, coarse_part;
  // finest level data for the right-hand side
  stgmg::LevelHost fine_info;  // sizes, Kcell (no matrices)
  stgmg::Material mat{};
  stgmg::TimeConsts T;
  stgmg::TimeBlockConsts tbc{};
  stgmg::TimeOp top{};
  bool tb = false;   // patch solves through the time eigen-decomposition
  bool red = false;  // ... with the u-equation rows eliminated
  DArr<double> e_dev, tmp_ns, src_buf;
  // time marching (stgmg_march): the slab start values at t_{n-1}, the slab's Radau times on the
  // device, and the right-hand side assembly captured as a graph (hierarchies with a V-cycle graph)
  DArr<double> xend, tdev;
  hipGraph_t rhs_graph = nullptr;
  hipGraphExec_t rhs_exec = nullptr;
  DevCsr cface;  // Problem B.1: boundary part of C on the finest level (right-hand side's jump)
  DArr<double> src_xq, src_wq, src_bq, src_bp, kfine;  // device source tables
  // kernel timing (finest level): event pairs per kernel class
  bool prof = false;
  std::vector<std::pair<hipEvent_t, hipEvent_t>> ev[2];
  size_t ev_used[2] = {0, 0};
  // FGMRES workspace
  int m_alloc = 0;
  DArr<double> V, Z, w, partials, hdev, ydev;
  double* hhost = nullptr;  // pinned, 512 doubles: Hessenberg column reads, then the FGMRES update coefficients at 256
  DArr<double> gin, gout;
  ~stgmg_handle() {
    if (graph_exec) (void)hipGraphExecDestroy(graph_exec);
    if (graph) (void)hipGraphDestroy(graph);
    if (rhs_exec) (void)hipGraphExecDestroy(rhs_exec);
    if (rhs_graph) (void)hipGraphDestroy(rhs_graph);
    if (enter_ev) (void)hipEventDestroy(enter_ev);
    for (auto e : vc_ev)
      if (e) (void)hipEventDestroy(e);
    if (hhost) (void)hipHostFree(hhost);
    for (auto& v : ev)
      for (auto& e : v) {
        (void)hipEventDestroy(e.first);
        (void)hipEventDestroy(e.second);
      }
  }
};

namespace {

using stgmg::LevelHost;

void vcycle(stgmg_handle* h, int l, const double* b, double* d);

// Order the handle's stream after the work enqueued on the caller's stream.
void enter(stgmg_handle* h) {
  HIPCHK(hipEventRecord(h->enter_ev, h->caller));
  HIPCHK(hipStreamWaitEvent(h->st, h->enter_ev, 0));
}

// Capture the finest-level V-cycle (gin -> gout) as a graph.  Called at the end of setup:
// while a stream captures, this runtime rejects null-stream work issued by other threads
// (and that work invalidates the capture), so the capture happens in the thread that sets the
// handle up, before the handle can be used from several threads.
void enqueue_slab_rhs(stgmg_handle* h, double t_start, const double* tdev, const double* x_prev_end_dev,
                      double* rhs_dev);

void capture_graph(stgmg_handle* h) {
  HIPCHK(hipStreamBeginCapture(h->st, hipStreamCaptureModeThreadLocal));
  vcycle(h, h->L, h->gin.p, h->gout.p);
  HIPCHK(hipStreamEndCapture(h->st, &h->graph));
  HIPCHK(hipGraphInstantiate(&h->graph_exec, h->graph, nullptr, nullptr, 0));
  // the slab right-hand side of time marching: xend -> src_buf, times read from tdev
  HIPCHK(hipStreamBeginCapture(h->st, hipStreamCaptureModeThreadLocal));
  enqueue_slab_rhs(h, 0.0, h->tdev.p, h->xend.p, h->src_buf.p);
  HIPCHK(hipStreamEndCapture(h->st, &h->rhs_graph));
  HIPCHK(hipGraphInstantiate(&h->rhs_exec, h->rhs_graph, nullptr, nullptr, 0));
}

// z = B r on the finest level: graph replay (through gin/gout) or direct launches.
void apply_B(stgmg_handle* h, const double* r, double* z) {
  if (!h->use_graph || h->prof) {
    vcycle(h, h->L, r, z);
    return;
  }
  const int64_t n = h->lv[h->L].n;
  if (!h->graph_exec) capture_graph(h);
  HIPCHK(hipMemcpyAsync(h->gin.p, r, n * sizeof(double), hipMemcpyDeviceToDevice, h->st));
  HIPCHK(hipGraphLaunch(h->graph_exec, h->st));
  HIPCHK(hipMemcpyAsync(z, h->gout.p, n * sizeof(double), hipMemcpyDeviceToDevice, h->st));
}

void check_params(const stgmg_params* p) {
  if (!p) throw ApiError(STGMG_ERR_INVALID_ARG, "params is NULL");
  if (p->dim != 2 && p->dim != 3) throw ApiError(STGMG_ERR_INVALID_ARG, "dim must be 2 or 3");
  if (p->coarse_cells < 1 || p->levels < 1 || p->levels > 12)
    throw ApiError(STGMG_ERR_INVALID_ARG, "coarse_cells >= 1 and 1 <= levels <= 12 required");
  if (p->r < 2 || p->r > 4) throw ApiError(STGMG_ERR_UNSUPPORTED, "r must be in 2..4");
  if (p->k < 0 || p->k > 3) throw ApiError(STGMG_ERR_UNSUPPORTED, "k must be in 0..3");
  if (p->patch != STGMG_PATCH_CELL && p->patch != STGMG_PATCH_VERTEX)
    throw ApiError(STGMG_ERR_INVALID_ARG, "unknown patch kind");
  if (p->smoother_prec != STGMG_FP64 && p->smoother_prec != STGMG_FP32 && p->smoother_prec != STGMG_BF16)
    throw ApiError(STGMG_ERR_INVALID_ARG, "unknown smoother precision");
  if (p->smoother_prec == STGMG_BF16 && p->time_blocks != 3)
    throw ApiError(STGMG_ERR_UNSUPPORTED, "BF16 storage needs the symmetric tiles (time_blocks = 3)");
  if (p->n_smooth < 0 || p->n_smooth > 64) throw ApiError(STGMG_ERR_INVALID_ARG, "n_smooth out of range");
  if (!(p->tau > 0) || !(p->rho > 0) || !(p->mu > 0) || !(p->c0 > 0) || !(p->alpha >= 0) ||
      !(p->lambda >= 0) || !(p->omega > 0))
    throw ApiError(STGMG_ERR_INVALID_ARG, "tau, rho, mu, c0, omega must be > 0; lambda, alpha >= 0");
  const int64_t Nf = int64_t(p->coarse_cells) << (p->levels - 1);
  if (Nf > 4096) throw ApiError(STGMG_ERR_UNSUPPORTED, "grid too fine");
  if (!p->K_cells && !(p->K > 0)) throw ApiError(STGMG_ERR_INVALID_ARG, "K must be > 0");
  if (p->time_blocks < 0 || p->time_blocks > 3) throw ApiError(STGMG_ERR_INVALID_ARG, "time_blocks must be 0..3");
  if (p->pressure != STGMG_PRESSURE_CONT && p->pressure != STGMG_PRESSURE_DISC)
    throw ApiError(STGMG_ERR_INVALID_ARG, "unknown pressure space");
  if (p->form != STGMG_FORM_V && p->form != STGMG_FORM_DTU) throw ApiError(STGMG_ERR_INVALID_ARG, "unknown formulation");
  if (p->waves_per_patch != 0 && p->waves_per_patch != 1 && p->waves_per_patch != 2 && p->waves_per_patch != 4)
    throw ApiError(STGMG_ERR_INVALID_ARG, "waves_per_patch must be 0, 1, 2 or 4");
  if (p->autotune != 0 && p->autotune != 1) throw ApiError(STGMG_ERR_INVALID_ARG, "autotune must be 0 or 1");
}

// A vector argument must be device (or managed) memory known to the runtime, 8-byte aligned.
void check_dev(const void* p, const char* what) {
  if (!p) throw ApiError(STGMG_ERR_INVALID_ARG, std::string(what) + " is NULL");
  if (reinterpret_cast<uintptr_t>(p) % sizeof(double) != 0)
    throw ApiError(STGMG_ERR_BAD_POINTER, std::string(what) + " is not 8-byte aligned");
  hipPointerAttribute_t a{};
  if (hipPointerGetAttributes(&a, p) != hipSuccess) {
    (void)hipGetLastError();  // the failed query must not surface in a later call
    throw ApiError(STGMG_ERR_BAD_POINTER, std::string(what) + " is not memory the HIP runtime knows");
  }
  if (a.type != hipMemoryTypeDevice && a.type != hipMemoryTypeManaged && !a.isManaged)
    throw ApiError(STGMG_ERR_BAD_POINTER, std::string(what) + " is not device memory");
}

int host_threads() {
  unsigned t = std::thread::hardware_concurrency();
  if (t == 0) t = 4;
  return int(std::min(t, 32u));
}

size_t lds_limit() {
  // dynamic LDS per block used by the inversion kernel; 64 KiB works on every
  // CDNA part without changing kernel attributes
  return 64 * 1024;
}

// LDS one workgroup may use on the current device (160 KiB on gfx950)
size_t lds_per_block() {
  int dev = 0, v = 0;
  if (hipGetDevice(&dev) != hipSuccess ||
      hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess)
    return 64 * 1024;
  return size_t(v);
}

void vcycle(stgmg_handle* h, int l, const double* b, double* d);

// Kernel that inverts the reduced blocks (the node mass block and the Schur complements):
// RED_INV_LDS  the whole matrix in LDS (workgroup kernel, complex blocks in complex arithmetic),
// RED_INV_MFMA the matrix in global memory, trailing updates on MFMA (complex arithmetic),
// RED_INV_PANEL the panel kernel on the 2x2-block real form of complex blocks (used when neither
//               of the others fits).
// STGMG_GJ_KERNEL = lds, mfma or panel selects a kernel where its blocks fit (comparisons).
enum { RED_INV_LDS = 0, RED_INV_MFMA = 1, RED_INV_PANEL = 2 };
constexpr int RED_INV_MFMA_ROWS = 64;
int red_inv_kernel(bool any_c, int max_nr, int max_nn) {
  const std::string e = std::getenv("STGMG_GJ_KERNEL") ? std::getenv("STGMG_GJ_KERNEL") : "";
  const bool mfma_fits = stgmg::gj_mfma_bytes(max_nr, any_c) <= lds_per_block() &&
                         stgmg::gj_mfma_bytes(max_nn, false) <= lds_per_block();
  const bool lds_fits = stgmg::gj_lds_kernel_bytes(max_nr, any_c) <= lds_per_block() &&
                        stgmg::gj_lds_kernel_bytes(max_nn, false) <= lds_per_block();
  if (e == "lds" && lds_fits) return RED_INV_LDS;
  if (e == "mfma" && mfma_fits) return RED_INV_MFMA;
  if (e == "panel") return RED_INV_PANEL;
  // Schur blocks above RED_INV_MFMA_ROWS rows go to the MFMA kernel even where they fit in LDS
  // (patch-solve setup phase, 32^3 dG(1) cell patches, 89 rows: 0.151 s in LDS, 0.125 s on MFMA;
  // 256^2 dG(2) vertex patches, 59 rows: 0.141 s in LDS, 0.234 s on MFMA)
  if (lds_fits && !(max_nr > RED_INV_MFMA_ROWS && mfma_fits)) return RED_INV_LDS;
  return mfma_fits ? RED_INV_MFMA : RED_INV_PANEL;
}
int red_inv_kernel(const stgmg::TimeBlockConsts& tb, int max_nr, int max_nn) {
  bool any_c = false;
  for (int a = 0; a < tb.nblk; ++a) any_c = any_c || tb.cplx[a];
  return red_inv_kernel(any_c, max_nr, max_nn);
}

// symmetric tiles need real kept eigenvalues > 0 (real square roots); true for dG(k)
bool red_sym_possible(const stgmg::TimeBlockConsts& tb) {
  for (int a = 0; a < tb.nblk; ++a)
    if (!tb.cplx[a] && !(tb.lam[2 * a] > 0.0)) return false;
  return true;
}

// stored 64-value tiles of the lower triangle of an nr x nr matrix (FP32: tiles paired)
// tiles interleaved per 8-byte unit of the stored values: 1 (FP64), 2 (FP32), 4 (BF16)
int tiles_per_unit(int32_t prec) { return prec == STGMG_BF16 ? 4 : prec == STGMG_FP32 ? 2 : 1; }
int64_t red_sym_tiles(int nr, int32_t prec) { return stgmg::sym_slots(nr, tiles_per_unit(prec)); }
size_t value_bytes(int32_t prec) { return prec == STGMG_BF16 ? 2 : prec == STGMG_FP32 ? 4 : 8; }

// FP32 storage takes the tiles up to this many Schur rows and the square layout beyond: one
// wave streams a patch's tiles, and with 4-byte values it keeps half the bytes of FP64 in
// flight (larger batches spill registers), while the square kernel splits the columns over
// several waves (measured FP32 patch kernels, tiles against square: 59 rows 0.744 / 0.842 ms,
// 89 rows 0.486 / 0.559 ms, 122 rows 1.089 / 0.770 ms, 402 rows 18.4 / 10.3 ms)
constexpr int FP32_SYM_MAX_NR = 96;
bool red_sym_used(const stgmg_params& p, bool sym_possible, int max_nr) {
  return p.time_blocks == 3 && sym_possible && (p.smoother_prec != STGMG_FP32 || max_nr <= FP32_SYM_MAX_NR);
  // (BF16 storage exists only as tiles: check_level_storage rejects a level without them)
}

// Event pair around one launch of kernel class `what` on the finest level.
struct ProfScope {
  stgmg_handle* h;
  int what;
  bool on;
  ProfScope(stgmg_handle* hh, int w, int level) : h(hh), what(w), on(hh->prof && level == hh->L) {
    if (!on) return;
    auto& v = h->ev[what];
    if (h->ev_used[what] == v.size()) {
      hipEvent_t a, b;
      HIPCHK(hipEventCreate(&a));
      HIPCHK(hipEventCreate(&b));
      v.emplace_back(a, b);
    }
    HIPCHK(hipEventRecord(v[h->ev_used[what]].first, h->st));
  }
  ~ProfScope() {
    if (on) (void)hipEventRecord(h->ev[what][h->ev_used[what]++].second, h->st);
  }
};

// Level operator: mode 0 y = A_l x, mode 1 y = b - A_l x (factored form).
void op_apply(stgmg_handle* h, int l, int mode, const double* x, const double* b, double* y) {
  const LevelDev& L = h->lv[l];
  if (L.node_ok) {
    stgmg::k_node_op(h->st, mode, h->top, L.node, L.ns, L.MMs.ptr.p, L.MMs.col.p, L.MMs.val.p, L.KKs.ptr.p,
                     L.KKs.col.p, L.KKs.val.p, x, b, y);
    return;
  }
  stgmg::k_kron_spmv(h->st, mode, h->top, L.ns, L.MMs.ptr.p, L.MMs.col.p, L.MMs.val.p, L.KKs.ptr.p, L.KKs.col.p,
                     L.KKs.val.p, x, b, y, L.op_lanes);
}

// The patch solves y_P = A_P^{-1} R_P r of one level, in the level's storage mode.
void launch_patch_apply(stgmg_handle* h, LevelDev& L, const double* r) {
  const bool f32 = h->prm.smoother_prec == STGMG_FP32;
  if (h->red && h->prm.smoother_prec == STGMG_BF16)
    stgmg::k_patch_apply_red_bf16(h->st, L.npatch, L.max_np, L.max_nu, L.max_nr, L.sym, L.waves, h->tbc, h->prm.dim,
                                  L.poff.p, L.pdof.p, L.tpos.p, L.pnu.p, L.ioff.p, L.inv16.p, r, L.y.p);
  else if (h->red && f32)
    stgmg::k_patch_apply_red_f32(h->st, L.npatch, L.max_np, L.max_nu, L.max_nr, L.sym, L.waves,
                                 h->tbc, h->prm.dim,
                                 L.poff.p, L.pdof.p, L.tpos.p, L.pnu.p, L.ioff.p, L.inv32.p, r, L.y.p);
  else if (h->red)
    stgmg::k_patch_apply_red_f64(h->st, L.npatch, L.max_np, L.max_nu, L.max_nr, L.sym, L.waves,
                                 h->tbc, h->prm.dim,
                                 L.poff.p, L.pdof.p, L.tpos.p, L.pnu.p, L.ioff.p, L.inv64.p, r, L.y.p);
  else if (h->tb && f32)
    stgmg::k_patch_apply_tb_f32(h->st, L.npatch, L.max_np, h->tbc, L.poff.p, L.pdof.p, L.tpos.p, L.ioff.p, L.inv32.p, r,
                                L.y.p);
  else if (h->tb)
    stgmg::k_patch_apply_tb_f64(h->st, L.npatch, L.max_np, h->tbc, L.poff.p, L.pdof.p, L.tpos.p, L.ioff.p, L.inv64.p, r,
                                L.y.p);
  else if (f32)
    stgmg::k_patch_apply_f32(h->st, L.npatch, L.max_np, L.poff.p, L.pdof.p, L.tpos.p, L.ioff.p, L.inv32.p, r, L.y.p);
  else
    stgmg::k_patch_apply_f64(h->st, L.npatch, L.max_np, L.poff.p, L.pdof.p, L.tpos.p, L.ioff.p, L.inv64.p, r, L.y.p);
}

// Autotuning (stgmg_params.autotune): on every smoothed level the candidate launch shapes are timed
// with HIP events (one warm-up and three timed launches each, on zero vectors) and the fastest is
// kept: the waves per patch of the tiled patch kernel (1, 2 or 4, unless waves_per_patch fixes it)
// and, on every level, the lanes per node of the operator kernel (2, 4, 8 or 16).
void autotune(stgmg_handle* h) {
  hipEvent_t e0, e1;
  HIPCHK(hipEventCreate(&e0));
  HIPCHK(hipEventCreate(&e1));
  auto time3 = [&](auto&& launch) {
    float ms = 0.f;
    for (int rep = 0; rep < 4; ++rep) {
      if (rep == 1) HIPCHK(hipEventRecord(e0, h->st));
      launch();
    }
    HIPCHK(hipEventRecord(e1, h->st));
    HIPCHK(hipEventSynchronize(e1));
    HIPCHK(hipEventElapsedTime(&ms, e0, e1));
    return ms;
  };
  for (int l = 0; l <= h->L; ++l) {
    LevelDev& L = h->lv[l];
    stgmg::k_fill_zero(h->st, L.r.p, L.n);
    stgmg::k_fill_zero(h->st, L.d.p, L.n);
    stgmg::k_fill_zero(h->st, L.b.p, L.n);
    if (L.sym && L.npatch > 0 && h->prm.waves_per_patch == 0) {
      float best = 0.f;
      int best_w = 1;
      for (int w : {1, 2, 4}) {
        L.waves = w;
        const float ms = time3([&] { launch_patch_apply(h, L, L.r.p); });
        if (w == 1 || ms < best) {
          best = ms;
          best_w = w;
        }
      }
      L.waves = best_w;
    }
    if (L.node_ok) {
      float best = 0.f;
      int best_g = 0;
      for (int g : {2, 4, 8, 16}) {
        L.node.lanes = g;
        const float ms = time3([&] { op_apply(h, l, 1, L.d.p, L.b.p, L.r.p); });
        if (best_g == 0 || ms < best) {
          best = ms;
          best_g = g;
        }
      }
      L.node.lanes = best_g;
    }
  }
  HIPCHK(hipGetLastError());
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
}

void smooth(stgmg_handle* h, int l, const double* b, double* d, int sweeps, bool zero_start) {
  LevelDev& L = h->lv[l];
  for (int j = 0; j < sweeps; ++j) {
    const double* r = b;
    if (!(j == 0 && zero_start)) {
      ProfScope ps(h, STGMG_PROF_RESIDUAL, l);
      op_apply(h, l, 1, d, b, L.r.p);
      r = L.r.p;
    }
    {
      ProfScope ps(h, STGMG_PROF_PATCH_APPLY, l);
      launch_patch_apply(h, L, r);
    }
    // a sweep from d = 0 writes d instead of adding to it (0 + x = x: the same values)
    stgmg::k_vanka_update(h->st, L.n, L.tptr.p, L.winv.p, L.y.p, d, j == 0 && zero_start);
  }
}

void vcycle(stgmg_handle* h, int l, const double* b, double* d) {
  if (l == 0) {
    stgmg::k_dense_gemv_t(h->st, h->n0, h->coarse_inv.p, b, h->coarse_part.p, d);
    return;
  }
  LevelDev& L = h->lv[l];
  LevelDev& C = h->lv[l - 1];
  const int J = h->prm.n_smooth;
  if (J == 0) stgmg::k_fill_zero(h->st, d, L.n);  // else the first sweep writes d
  smooth(h, l, b, d, J, true);
  op_apply(h, l, 1, d, b, L.r.p);
  L.R.apply(h->st, 0, L.r.p, nullptr, C.b.p);
  vcycle(h, l - 1, C.b.p, C.d.p);
  L.P.apply(h->st, 2, C.d.p, nullptr, d);
  smooth(h, l, b, d, J, false);
}

// Dense transposed copy of a CSR matrix: W[c * n + r] = A[r][c].
std::vector<double> dense_transposed(const stgmg::Csr& A) {
  const int64_t n = A.nrows;
  std::vector<double> W(size_t(n) * n, 0.0);
  for (int64_t r = 0; r < n; ++r)
    for (int64_t p = A.ptr[r]; p < A.ptr[r + 1]; ++p) W[size_t(A.col[p]) * n + r] = A.val[p];
  return W;
}

// Test hook: STGMG_TEST_ZERO_PATCH=q zeroes the first block that the setup inverts for patch q of
// the finest level (the node mass block of the reduced solves, the whole A_P of the full
// inverses, the first time block otherwise), so that the inversion meets a zero pivot and
// stgmg_setup returns STGMG_ERR_SINGULAR_PATCH.  Unset in normal use.
int64_t test_zero_patch() {
  const char* e = std::getenv("STGMG_TEST_ZERO_PATCH");
  return e ? std::atoll(e) : -1;
}

// Wall time of the setup phases (host assembly, node-pair extraction, coarse inverse, transfers,
// patch solves), printed to stderr when STGMG_SETUP_TIMES is set.
struct SetupClock {
  using C = std::chrono::steady_clock;
  C::time_point t = C::now();
  double sec[5] = {0, 0, 0, 0, 0};  // assembly, node pairs, coarse, transfers, patch solves
  void lap(int phase) {
    const C::time_point u = C::now();
    sec[phase] += std::chrono::duration<double>(u - t).count();
    t = u;
  }
};

void build(stgmg_handle* h) {
  const stgmg_params& p = h->prm;
  const int64_t zero_patch = test_zero_patch();
  SetupClock clk;
  const int d = p.dim, L = p.levels - 1;
  h->L = L;
  h->mat = {p.rho, p.lambda, p.mu, p.alpha, p.c0};
  h->T = stgmg::make_time_consts(p.k, p.tau);
  h->tb = p.time_blocks != 0;
  h->red = p.time_blocks >= 2;
  h->top.nt = p.k + 1;
  for (int b = 0; b <= p.k; ++b) {
    h->top.mt[b] = h->T.mt[b];
    for (int a = 0; a <= p.k; ++a) h->top.D[b * (p.k + 1) + a] = h->T.Dt[b * (p.k + 1) + a];
  }
  if (h->tb) {
    const stgmg::TimeBlocks B = stgmg::make_time_blocks(h->T);
    h->tbc.nt = B.nt;
    h->tbc.nblk = B.nblk;
    for (int a = 0; a < B.nblk; ++a) {
      h->tbc.lam[2 * a] = B.lam[a].real();
      h->tbc.lam[2 * a + 1] = B.lam[a].imag();
      h->tbc.cplx[a] = B.is_complex[a];
      for (int b = 0; b < B.nt; ++b) {
        h->tbc.tin[2 * (a * B.nt + b)] = B.tin[a * B.nt + b].real();
        h->tbc.tin[2 * (a * B.nt + b) + 1] = B.tin[a * B.nt + b].imag();
      }
    }
    for (int b = 0; b < B.nt; ++b)
      for (int a = 0; a < B.nblk; ++a) {
        h->tbc.qout[2 * (b * B.nblk + a)] = B.qout[b * B.nblk + a].real();
        h->tbc.qout[2 * (b * B.nblk + a) + 1] = B.qout[b * B.nblk + a].imag();
      }
  }
  const int nth = host_threads();
  int64_t* ctr = &h->bytes;
  // permeability per level: finest from the caller, coarse = mean of the 2^d children
  std::vector<std::vector<double>> Kl(L + 1);
  {
    const int Nf = p.coarse_cells << L;
    int64_t nc = 1;
    for (int a = 0; a < d; ++a) nc *= Nf;
    Kl[L].assign(nc, p.K);
    if (p.K_cells) {
      for (int64_t c = 0; c < nc; ++c) {
        if (!(p.K_cells[c] > 0) || !std::isfinite(p.K_cells[c]))
          throw ApiError(STGMG_ERR_INVALID_ARG, "K_cells must be finite and > 0");
        Kl[L][c] = p.K_cells[c];
      }
    }
    for (int l = L - 1; l >= 0; --l) {
      const int N = p.coarse_cells << l;
      int64_t ncl = 1;
      for (int a = 0; a < d; ++a) ncl *= N;
      Kl[l].assign(ncl, 0.0);
      const int Nfn = 2 * N;
      for (int64_t c = 0; c < ncl; ++c) {
        int cc[3] = {0, 0, 0};
        int64_t rem = c;
        for (int a = 0; a < d; ++a) {
          cc[a] = int(rem % N);
          rem /= N;
        }
        double s = 0.0;
        for (int ch = 0; ch < (1 << d); ++ch) {
          int64_t idx = 0;
          for (int a = d - 1; a >= 0; --a) idx = idx * Nfn + (2 * cc[a] + ((ch >> a) & 1));
          s += Kl[l + 1][idx];
        }
        Kl[l][c] = s / double(1 << d);
      }
    }
  }
  h->lv.resize(L + 1);
  LevelHost prev;
  for (int l = 0; l <= L; ++l) {
    LevelHost H;
    stgmg::BuildOptions o{d, p.r, p.k, p.coarse_cells << l, p.patch, p.tau, p.omega, l >= 1, true, true,
                          l == 0 || !h->tb, p.pressure == STGMG_PRESSURE_DISC, p.form == STGMG_FORM_DTU,
                          p.form == STGMG_FORM_DTU && l == L};
    stgmg::build_level(o, h->mat, Kl[l], H, nth);
    clk.lap(0);
    LevelDev& D = h->lv[l];
    D.N = H.N;
    D.n = H.n;
    D.ns = H.ns;
    if (l >= 1 && !h->tb) D.A.upload(H.A, h->st, ctr);  // full-inverse patch extraction reads it
    D.MMs.upload(H.MM, h->st, ctr);
    D.KKs.upload(H.KK, h->st, ctr);
    D.alg_op_values = double(H.MM.col.size() + H.KK.col.size());
    {
      stgmg::NodeOp no;
      if (stgmg::build_node_op(H, no, nth)) {
        D.nptr.upload(no.ptr, h->st, ctr);
        D.ncol.upload(no.col, h->st, ctr);
        D.nm.upload(no.m, h->st, ctr);
        D.na.upload(no.a, h->st, ctr);
        D.ncptr.upload(no.cptr, h->st, ctr);
        D.nccol.upload(no.ccol, h->st, ctr);
        D.nc.upload(no.c, h->st, ctr);
        D.node = {d, no.nQ, 0, D.nptr.p, D.ncol.p, D.nm.p, D.na.p, D.ncptr.p, D.nccol.p, D.nc.p};
        D.node_ok = true;
        // pressure rows from the CSRs, velocity rows from the node pairs
        const int64_t pr0 = 2 * H.nv;
        D.alg_op_values = double(no.m.size() + no.a.size() + no.c.size()) +
                          double(H.MM.ptr[H.ns] - H.MM.ptr[pr0] + H.KK.ptr[H.ns] - H.KK.ptr[pr0]);
        HIPCHK(hipStreamSynchronize(h->st));  // the host arrays of `no` are freed at the end of this block
      }
      clk.lap(1);
    }
    if (l == L && p.form == STGMG_FORM_DTU) h->cface.upload(H.Cface, h->st, ctr);
    {
      const double avg = H.ns ? double(H.MM.col.size() + H.KK.col.size()) / double(H.ns) : 0.0;
      D.op_lanes = avg < 12 ? 4 : 8;  // 8 lanes per spatial row measured best on the 256^2 dG(2) operator
      if (const char* e = std::getenv("STGMG_OP_LANES")) {  // tuning override
        const int v = std::atoi(e);
        if (v == 4 || v == 8 || v == 16 || v == 32) D.op_lanes = std::max(v, p.k + 1);
      }
      D.op_lanes = std::max(D.op_lanes, 4);
    }
    D.b.alloc(H.n, ctr, h->st);
    D.d.alloc(H.n, ctr, h->st);
    D.r.alloc(H.n, ctr, h->st);
    if (l == 0) {
      if (H.n > 20000) throw ApiError(STGMG_ERR_UNSUPPORTED, "coarsest level too large for the dense inverse");
      h->n0 = int(H.n);
      std::vector<double> W0 = dense_transposed(H.A);
      DArr<double> Wd;
      Wd.upload(W0, h->st, nullptr);  // W0 (pageable) stays alive until the synchronisation below
      h->coarse_inv.alloc(H.n * stgmg::inv_ld(int(H.n)), ctr, h->st);
      h->coarse_part.alloc(int64_t(stgmg::dense_gemv_chunks(int(H.n))) * H.n, ctr, h->st);
      DArr<int32_t> stat;
      const std::vector<int32_t> stat0(1, 0);
      stat.upload(stat0, h->st, nullptr);
      // one workgroup for small matrices; above a few hundred rows the panel steps over many
      // workgroups win (1047 rows: 357 ms in one workgroup)
      const int nb = H.n <= 384 ? stgmg::gj_panel_width(int(H.n), lds_limit()) : 0;
      if (nb != 0) {
        // one workgroup holds the whole inversion
        const int n0 = int(H.n);
        const std::vector<stgmg::GjDesc> d0 = {{n0, n0, stgmg::inv_ld(n0), 0, 0, 0, 0, 0}};
        DArr<stgmg::GjDesc> dd;
        dd.upload(d0, h->st, nullptr);
        stgmg::k_gj_invert_f64(h->st, nb, 1, n0, dd.p, Wd.p, h->coarse_inv.p, stat.p);
        HIPCHK(hipGetLastError());
        HIPCHK(hipStreamSynchronize(h->st));
      } else {
        // panels over many workgroups
        const int n0 = int(H.n), pnb = 32;
        DArr<double> scl, Wb, P0, P1;
        DArr<int> perm, src;
        scl.alloc(n0, nullptr, h->st);
        Wb.alloc(int64_t(pnb) * n0, nullptr, h->st);
        P0.alloc(int64_t(pnb) * n0, nullptr, h->st);
        P1.alloc(int64_t(pnb) * n0, nullptr, h->st);
        perm.alloc(n0, nullptr, h->st);
        src.alloc(n0, nullptr, h->st);
        stgmg::k_gj_large_rowscale(h->st, n0, Wd.p, scl.p);
        for (int k0 = 0; k0 < n0; k0 += pnb)
          stgmg::k_gj_large_step(h->st, n0, k0, std::min(pnb, n0 - k0), Wd.p, perm.p, P0.p, P1.p, Wb.p, stat.p);
        HIPCHK(hipGetLastError());
        std::vector<int> perm_h(n0), src_h(n0);
        HIPCHK(hipMemcpyAsync(perm_h.data(), perm.p, n0 * sizeof(int), hipMemcpyDeviceToHost, h->st));
        HIPCHK(hipStreamSynchronize(h->st));
        for (int j = 0; j < n0; ++j) src_h[j] = j;
        for (int k = n0 - 1; k >= 0; --k) std::swap(src_h[k], src_h[perm_h[k]]);
        HIPCHK(hipMemcpyAsync(src.p, src_h.data(), n0 * sizeof(int), hipMemcpyHostToDevice, h->st));
        stgmg::k_gj_large_output(h->st, n0, Wd.p, src.p, scl.p, h->coarse_inv.p);
        HIPCHK(hipGetLastError());
        HIPCHK(hipStreamSynchronize(h->st));
      }
      int32_t s = 0;
      HIPCHK(hipMemcpyAsync(&s, stat.p, sizeof(int32_t), hipMemcpyDeviceToHost, h->st));
      HIPCHK(hipStreamSynchronize(h->st));
      if (s) throw ApiError(STGMG_ERR_SINGULAR_PATCH, "coarse operator is singular");
      clk.lap(2);
    }
    if (l >= 1) {
      stgmg::Csr P = stgmg::build_prolongation(prev, H, nth);
      D.P.upload(P, h->st, ctr);
      {
        // P is block diagonal over (time node, field): V, U, P rows of each fine time node
        // interpolate from the same block of the coarse time node
        std::vector<int64_t> rb{0}, cb{0};
        for (int tn = 0; tn <= p.k; ++tn)
          for (int f = 0; f < 3; ++f) {
            rb.push_back(tn * H.ns + (f == 0 ? H.nv : f == 1 ? 2 * H.nv : H.ns));
            cb.push_back(tn * prev.ns + (f == 0 ? prev.nv : f == 1 ? 2 * prev.nv : prev.ns));
          }
        D.R.upload(stgmg::transpose_block_diag(P, H.n, rb, cb, nth), h->st, ctr);
      }
      HIPCHK(hipStreamSynchronize(h->st));
      clk.lap(3);
      // patches
      D.npatch = H.npatch;
      D.poff_h = H.poff;
      D.pdof_h = H.pdof;
      D.ioff_h.assign(H.npatch + 1, 0);
      int max_np = 0;
      int red_kernel = RED_INV_LDS;
      if (h->red) {
        D.pnu_h.assign(H.npatch, 0);
        for (int64_t q = 0; q < H.npatch; ++q) {
          // time node 0 of the patch: V dofs (spatial numbers < nv), U dofs, P dofs
          const int64_t ns = (H.poff[q + 1] - H.poff[q]) / (p.k + 1);
          int64_t nU = 0;
          for (int64_t t = 0; t < ns; ++t) nU += H.pdof[H.poff[q] + t] < H.nv ? 1 : 0;
          const int64_t nP = ns - 2 * nU, nr = nU + nP;
          if (nU % d != 0 || nP < 0) throw ApiError(STGMG_ERR_HIP, "unexpected patch layout");
          D.pnu_h[q] = int32_t(nU);
          D.max_nu = std::max<int>(D.max_nu, int(nU));
          D.max_nr = std::max<int>(D.max_nr, int(nr));
          D.max_npr = std::max<int>(D.max_npr, int(nP));
        }
        red_kernel = red_inv_kernel(h->tbc, D.max_nr, D.max_nu / d);
        D.sym = red_sym_used(p, red_sym_possible(h->tbc), D.max_nr);
      }
      for (int64_t q = 0; q < H.npatch; ++q) {
        const int64_t np = H.poff[q + 1] - H.poff[q];
        max_np = std::max<int>(max_np, int(np));
        if (h->red) {
          const int64_t ns = np / (p.k + 1), nU = D.pnu_h[q];
          const int64_t nP = ns - 2 * nU, nn = nU / d, nr = nU + nP;
          int64_t sz = nn * stgmg::inv_ld(int(nn)) + nU * stgmg::inv_ld(int(nP));
          D.alg_inv_entries += double(nn * nn + nP * nU);
          for (int a = 0; a < h->tbc.nblk; ++a) {
            const int64_t planes = h->tbc.cplx[a] ? 2 : 1;
            if (D.sym) {
              sz += planes * red_sym_tiles(int(nr), p.smoother_prec) * 64;
              D.alg_inv_entries += double(planes * nr * (nr + 1) / 2);
            } else {
              sz += planes * nr * stgmg::inv_ld(int(nr));
              D.alg_inv_entries += double(planes * nr * nr);
            }
          }
          D.ioff_h[q + 1] = D.ioff_h[q] + sz;
        } else if (h->tb) {
          const int64_t ns = np / (p.k + 1), ldh = stgmg::inv_ld(int(ns));
          int64_t sz = 0;
          for (int a = 0; a < h->tbc.nblk; ++a) {
            sz += h->tbc.cplx[a] ? ns * 2 * ldh : ns * ldh;
            D.alg_inv_entries += double(h->tbc.cplx[a] ? 2 * ns * ns : ns * ns);
          }
          D.ioff_h[q + 1] = D.ioff_h[q] + sz;
        } else {
          D.ioff_h[q + 1] = D.ioff_h[q] + np * stgmg::inv_ld(int(np));
          D.alg_inv_entries += double(np * np);
        }
      }
      D.max_np = max_np;
      D.poff.upload(H.poff, h->st, ctr);
      D.pdof.upload(H.pdof, h->st, ctr);
      D.ioff.upload(D.ioff_h, h->st, ctr);
      if (h->red) D.pnu.upload(D.pnu_h, h->st, ctr);
      D.tptr.upload(H.tptr, h->st, ctr);
      if (H.tpos.size() >= (size_t(1) << 31)) throw ApiError(STGMG_ERR_UNSUPPORTED, "too many patch entries");
      D.tpos.upload(H.tpos, h->st, ctr);
      D.winv.upload(H.winv, h->st, ctr);
      D.y.alloc(int64_t(H.pdof.size()), ctr, h->st);
      const int64_t tot = D.ioff_h[H.npatch];
      if (p.smoother_prec == STGMG_BF16 && !D.sym)
        throw ApiError(STGMG_ERR_UNSUPPORTED, "BF16 storage needs the symmetric tiles (positive real eigenvalues)");
      if (p.smoother_prec == STGMG_BF16)
        D.inv16.alloc(tot, ctr, h->st);
      else if (p.smoother_prec == STGMG_FP32)
        D.inv32.alloc(tot, ctr, h->st);
      else
        D.inv64.alloc(tot, ctr, h->st);
      DArr<int32_t> stat;
      const std::vector<int32_t> stat0(H.npatch, 0);
      stat.upload(stat0, h->st, nullptr);
      if (!h->tb) {
        // full space-time inverses: extraction + inversion in batches through a dense work buffer
        const int nb = stgmg::gj_panel_width(max_np, lds_limit());
        if (nb == 0) throw ApiError(STGMG_ERR_UNSUPPORTED, "patch too large for the inversion kernel");
        const int64_t stride = int64_t(max_np) * max_np;
        int64_t batch = std::max<int64_t>(1, std::min<int64_t>(H.npatch, (int64_t(3) << 30) / (stride * 8)));
        DArr<double> Wb;
        Wb.alloc(batch * stride, nullptr, h->st);
        std::vector<int64_t> woff_h(batch);
        for (int64_t i = 0; i < batch; ++i) woff_h[i] = i * stride;
        DArr<int64_t> woff;
        woff.upload(woff_h, h->st, nullptr);
        std::vector<std::vector<stgmg::GjDesc>> descs;
        std::vector<DArr<stgmg::GjDesc>> ddesc;
        for (int64_t p0 = 0; p0 < H.npatch; p0 += batch) {
          const int64_t cnt = std::min(batch, H.npatch - p0);
          std::vector<stgmg::GjDesc> dd(cnt);
          for (int64_t i = 0; i < cnt; ++i) {
            const int np = int(H.poff[p0 + i + 1] - H.poff[p0 + i]);
            dd[i] = {np, np, stgmg::inv_ld(np), 0, 0, int32_t(p0 + i), i * stride, D.ioff_h[p0 + i]};
          }
          descs.push_back(std::move(dd));
          ddesc.emplace_back();
          ddesc.back().upload(descs.back(), h->st, nullptr);
          stgmg::k_fill_zero(h->st, Wb.p, cnt * stride);
          stgmg::k_patch_extract_t(h->st, p0, cnt, max_np, D.poff.p, D.pdof.p, D.A.ptr.p, D.A.col.p, D.A.val.p,
                                   woff.p, Wb.p);
          if (l == L && zero_patch >= p0 && zero_patch < p0 + cnt)
            stgmg::k_fill_zero(h->st, Wb.p + (zero_patch - p0) * stride, stride);
          if (p.smoother_prec == STGMG_FP32)
            stgmg::k_gj_invert_f32(h->st, nb, cnt, max_np, ddesc.back().p, Wb.p, D.inv32.p, stat.p);
          else
            stgmg::k_gj_invert_f64(h->st, nb, cnt, max_np, ddesc.back().p, Wb.p, D.inv64.p, stat.p);
          HIPCHK(hipGetLastError());
        }
        HIPCHK(hipStreamSynchronize(h->st));
      } else if (h->red) {
        // reduced time-block inverses: spatial MM_P, KK_P -> node mass block and one Schur
        // complement per kept eigenvalue (real or 2x2-block complex) -> batched Gauss-Jordan;
        // the (p-equation, V) block of KK_P is copied into the stored layout by the form kernel
        // and multiplied by the mass inverse after the inversion
        const int nt = p.k + 1, nblk = h->tbc.nblk;
        const int max_ns = max_np / nt, max_nr = D.max_nr, max_nn = D.max_nu / d;
        bool any_c = false;
        for (int a = 0; a < nblk; ++a) any_c = any_c || h->tbc.cplx[a];
        // blocks held entirely in LDS when they fit in one workgroup's LDS, else in global memory
        // with MFMA updates (both in complex arithmetic for complex blocks: real and imaginary
        // planes), else the panel kernel on the 2x2-block real form
        const bool in_lds = red_kernel == RED_INV_LDS, planes = red_kernel != RED_INV_PANEL;
        (void)any_c;
        int64_t per_patch = int64_t(max_nn) * max_nn;
        std::vector<int64_t> blk_woff(nblk);
        for (int a = 0; a < nblk; ++a) {
          blk_woff[a] = per_patch;
          const bool c = h->tbc.cplx[a] != 0;
          per_patch += planes ? (c ? 2 : 1) * int64_t(max_nr) * max_nr : (c ? 4 : 1) * int64_t(max_nr) * max_nr;
        }
        const int max_n = std::max(any_c ? 2 * max_nr : max_nr, max_nn);
        const int nb = planes ? 32 : stgmg::gj_panel_width(max_n, lds_limit());
        if (nb == 0) throw ApiError(STGMG_ERR_UNSUPPORTED, "patch too large for the inversion kernel");
        if (stgmg::patch_apply_red_threads(max_nr, p.smoother_prec == STGMG_FP32) > 512 || D.max_nu > 64 * 32)
          throw ApiError(STGMG_ERR_UNSUPPORTED, "patch too large for the reduced patch solve");
        const int64_t sq = int64_t(max_ns) * max_ns;
        // symmetric tiles: the Schur blocks are inverted into a square FP64 scratch per batch
        // item and packed from there
        int64_t sq_item = 0;
        if (D.sym)
          for (int a = 0; a < nblk; ++a) sq_item += (h->tbc.cplx[a] ? 2 : 1) * int64_t(max_nr) * stgmg::inv_ld(max_nr);
        const int64_t batch = std::max<int64_t>(
            1, std::min<int64_t>(H.npatch, (int64_t(3) << 30) / ((per_patch + 2 * sq + sq_item) * 8)));
        DArr<double> Wb, wmm, wkk, Sq;
        Wb.alloc(batch * per_patch, nullptr, h->st);
        wmm.alloc(batch * sq, nullptr, h->st);
        wkk.alloc(batch * sq, nullptr, h->st);
        if (D.sym) Sq.alloc(batch * sq_item, nullptr, h->st);
        std::vector<std::vector<stgmg::GjDesc>> descs;
        std::vector<std::vector<int32_t>> nss, nus, nrs;
        std::vector<std::vector<int64_t>> soffs, toffs;
        std::vector<DArr<stgmg::GjDesc>> ddesc;
        std::vector<DArr<int32_t>> dns, dnu, dnr;
        std::vector<DArr<int64_t>> dsoff, dtoff;
        for (int64_t p0 = 0; p0 < H.npatch; p0 += batch) {
          const int64_t cnt = std::min(batch, H.npatch - p0);
          std::vector<stgmg::GjDesc> dd(cnt * (nblk + 1));
          std::vector<int32_t> ns_of(cnt), nu_of(cnt), nr_of(cnt);
          std::vector<int64_t> soff(D.sym ? cnt * nblk : 0), toff(D.sym ? cnt * nblk : 0);
          for (int64_t i = 0; i < cnt; ++i) {
            const int ns = int(H.poff[p0 + i + 1] - H.poff[p0 + i]) / nt, nU = D.pnu_h[p0 + i];
            const int nP = ns - 2 * nU, nn = nU / d, nr = nU + nP;
            const int ldn = stgmg::inv_ld(nn), ldp = stgmg::inv_ld(nP), ldr = stgmg::inv_ld(nr);
            ns_of[i] = ns;
            nu_of[i] = nU;
            nr_of[i] = nr;
            int64_t oo = D.ioff_h[p0 + i];
            dd[i * (nblk + 1)] = {nn, nn, ldn, 0, 0, int32_t(p0 + i), i * per_patch, oo};
            oo += int64_t(nn) * ldn + int64_t(nU) * ldp;
            int64_t so = i * sq_item;
            for (int a = 0; a < nblk; ++a) {
              const bool c = h->tbc.cplx[a] != 0;
              const int n_in = c && !planes ? 2 * nr : nr;  // LDS and MFMA kernels: complex n x n
              dd[i * (nblk + 1) + 1 + a] = {n_in, nr, c ? 2 * ldr : ldr, c ? nr : 0, ldr,
                                            int32_t(p0 + i), i * per_patch + blk_woff[a], D.sym ? so : oo};
              if (D.sym) {
                soff[i * nblk + a] = so;
                toff[i * nblk + a] = oo;
                so += int64_t(nr) * (c ? 2 * ldr : ldr);
                oo += (c ? 2 : 1) * red_sym_tiles(nr, p.smoother_prec) * 64;
              } else {
                oo += int64_t(nr) * (c ? 2 * ldr : ldr);
              }
            }
          }
          // descriptors grouped by kernel for the LDS path, and by destination for the symmetric
          // tiles (mass blocks into the stored layout, Schur blocks into the scratch): mass
          // blocks, real blocks, complex blocks
          std::vector<stgmg::GjDesc> grp;
          int64_t n_mass = 0, n_real = 0;
          if (planes || D.sym) {
            for (int g = 0; g < 3; ++g)
              for (int64_t i = 0; i < cnt; ++i)
                for (int sl = 0; sl <= nblk; ++sl) {
                  const int kind = sl == 0 ? 0 : h->tbc.cplx[sl - 1] ? 2 : 1;
                  if (kind == g) grp.push_back(dd[i * (nblk + 1) + sl]);
                }
            n_mass = cnt;
            for (int a = 0; a < nblk; ++a) n_real += h->tbc.cplx[a] ? 0 : cnt;
          }
          const int64_t n_cplx = int64_t(grp.size()) - n_mass - n_real;
          descs.push_back(std::move(dd));
          descs.push_back(std::move(grp));
          nss.push_back(std::move(ns_of));
          nus.push_back(std::move(nu_of));
          ddesc.emplace_back();
          ddesc.back().upload(descs[descs.size() - 2], h->st, nullptr);
          ddesc.emplace_back();
          if (planes || D.sym) ddesc.back().upload(descs.back(), h->st, nullptr);
          const stgmg::GjDesc* dper = ddesc[ddesc.size() - 2].p;
          const stgmg::GjDesc* dgrp = ddesc.back().p;
          dns.emplace_back();
          dns.back().upload(nss.back(), h->st, nullptr);
          dnu.emplace_back();
          dnu.back().upload(nus.back(), h->st, nullptr);
          if (D.sym) {
            nrs.push_back(std::move(nr_of));
            soffs.push_back(std::move(soff));
            toffs.push_back(std::move(toff));
            dnr.emplace_back();
            dnr.back().upload(nrs.back(), h->st, nullptr);
            dsoff.emplace_back();
            dsoff.back().upload(soffs.back(), h->st, nullptr);
            dtoff.emplace_back();
            dtoff.back().upload(toffs.back(), h->st, nullptr);
          }
          stgmg::k_fill_zero(h->st, wmm.p, cnt * sq);
          stgmg::k_fill_zero(h->st, wkk.p, cnt * sq);
          stgmg::k_patch_extract_spatial_t(h->st, p0, cnt, nt, max_ns, D.poff.p, D.pdof.p, D.MMs.ptr.p, D.MMs.col.p,
                                           D.MMs.val.p, D.KKs.ptr.p, D.KKs.col.p, D.KKs.val.p, wmm.p, wkk.p);
          // the batched inversion of the planar layout: LDS or MFMA kernel
          auto gj64 = [&](bool c, int64_t m, int mx, const stgmg::GjDesc* dsc, double* o) {
            if (in_lds)
              stgmg::k_gj_lds_f64(h->st, c, m, mx, dsc, Wb.p, o, stat.p);
            else
              stgmg::k_gj_mfma_f64(h->st, c, m, mx, dsc, Wb.p, o, stat.p);
          };
          auto gj32 = [&](bool c, int64_t m, int mx, const stgmg::GjDesc* dsc, float* o) {
            if (in_lds)
              stgmg::k_gj_lds_f32(h->st, c, m, mx, dsc, Wb.p, o, stat.p);
            else
              stgmg::k_gj_mfma_f32(h->st, c, m, mx, dsc, Wb.p, o, stat.p);
          };
          auto gj16 = [&](bool c, int64_t m, int mx, const stgmg::GjDesc* dsc, __bf16* o) {
            if (in_lds)
              stgmg::k_gj_lds_bf16(h->st, c, m, mx, dsc, Wb.p, o, stat.p);
            else
              stgmg::k_gj_mfma_bf16(h->st, c, m, mx, dsc, Wb.p, o, stat.p);
          };
          if (p.smoother_prec == STGMG_BF16) {  // symmetric tiles only
            stgmg::k_form_reduced_blocks_bf16(h->st, cnt, h->tbc, d, planes ? 1 : 0, max_ns, max_nr, dns.back().p,
                                              dnu.back().p, wmm.p, wkk.p, dper, Wb.p, D.inv16.p);
            if (l == L && zero_patch >= p0 && zero_patch < p0 + cnt)
              stgmg::k_fill_zero(h->st, Wb.p + (zero_patch - p0) * per_patch, int64_t(max_nn) * max_nn);
            if (planes) {
              gj16(false, n_mass, max_nn, dgrp, D.inv16.p);
              gj64(false, n_real, max_nr, dgrp + n_mass, Sq.p);
              gj64(true, n_cplx, max_nr, dgrp + n_mass + n_real, Sq.p);
            } else {
              stgmg::k_gj_invert_bf16(h->st, nb, n_mass, max_n, dgrp, Wb.p, D.inv16.p, stat.p);
              stgmg::k_gj_invert_f64(h->st, nb, n_real + n_cplx, max_n, dgrp + n_mass, Wb.p, Sq.p, stat.p);
            }
            stgmg::k_pack_red_sym_bf16(h->st, cnt, h->tbc, dnu.back().p, dnr.back().p, dsoff.back().p,
                                       dtoff.back().p, Sq.p, D.inv16.p);
            stgmg::k_fold_reduced_bf16(h->st, cnt, d, D.max_nu, D.max_npr, dns.back().p, dnu.back().p, dper, nblk + 1,
                                       D.inv16.p);
          } else if (p.smoother_prec == STGMG_FP32) {
            stgmg::k_form_reduced_blocks_f32(h->st, cnt, h->tbc, d, planes ? 1 : 0, max_ns, max_nr, dns.back().p,
                                             dnu.back().p, wmm.p, wkk.p, dper, Wb.p, D.inv32.p);
            if (l == L && zero_patch >= p0 && zero_patch < p0 + cnt)
              stgmg::k_fill_zero(h->st, Wb.p + (zero_patch - p0) * per_patch, int64_t(max_nn) * max_nn);
            if (planes && D.sym) {
              gj32(false, n_mass, max_nn, dgrp, D.inv32.p);
              gj64(false, n_real, max_nr, dgrp + n_mass, Sq.p);
              gj64(true, n_cplx, max_nr, dgrp + n_mass + n_real, Sq.p);
              stgmg::k_pack_red_sym_f32(h->st, cnt, h->tbc, dnu.back().p, dnr.back().p, dsoff.back().p,
                                        dtoff.back().p, Sq.p, D.inv32.p);
            } else if (D.sym) {
              stgmg::k_gj_invert_f32(h->st, nb, n_mass, max_n, dgrp, Wb.p, D.inv32.p, stat.p);
              stgmg::k_gj_invert_f64(h->st, nb, n_real + n_cplx, max_n, dgrp + n_mass, Wb.p, Sq.p, stat.p);
              stgmg::k_pack_red_sym_f32(h->st, cnt, h->tbc, dnu.back().p, dnr.back().p, dsoff.back().p,
                                        dtoff.back().p, Sq.p, D.inv32.p);
            } else if (planes) {
              gj32(false, n_mass, max_nn, dgrp, D.inv32.p);
              gj32(false, n_real, max_nr, dgrp + n_mass, D.inv32.p);
              gj32(true, n_cplx, max_nr, dgrp + n_mass + n_real, D.inv32.p);
            } else {
              stgmg::k_gj_invert_f32(h->st, nb, cnt * (nblk + 1), max_n, dper, Wb.p, D.inv32.p, stat.p);
            }
            stgmg::k_fold_reduced_f32(h->st, cnt, d, D.max_nu, D.max_npr, dns.back().p, dnu.back().p, dper, nblk + 1,
                                      D.inv32.p);
          } else {
            stgmg::k_form_reduced_blocks_f64(h->st, cnt, h->tbc, d, planes ? 1 : 0, max_ns, max_nr, dns.back().p,
                                             dnu.back().p, wmm.p, wkk.p, dper, Wb.p, D.inv64.p);
            if (l == L && zero_patch >= p0 && zero_patch < p0 + cnt)
              stgmg::k_fill_zero(h->st, Wb.p + (zero_patch - p0) * per_patch, int64_t(max_nn) * max_nn);
            if (planes && D.sym) {
              gj64(false, n_mass, max_nn, dgrp, D.inv64.p);
              gj64(false, n_real, max_nr, dgrp + n_mass, Sq.p);
              gj64(true, n_cplx, max_nr, dgrp + n_mass + n_real, Sq.p);
              stgmg::k_pack_red_sym_f64(h->st, cnt, h->tbc, dnu.back().p, dnr.back().p, dsoff.back().p,
                                        dtoff.back().p, Sq.p, D.inv64.p);
            } else if (planes) {
              gj64(false, n_mass, max_nn, dgrp, D.inv64.p);
              gj64(false, n_real, max_nr, dgrp + n_mass, D.inv64.p);
              gj64(true, n_cplx, max_nr, dgrp + n_mass + n_real, D.inv64.p);
            } else if (D.sym) {
              stgmg::k_gj_invert_f64(h->st, nb, n_mass, max_n, dgrp, Wb.p, D.inv64.p, stat.p);
              stgmg::k_gj_invert_f64(h->st, nb, n_real + n_cplx, max_n, dgrp + n_mass, Wb.p, Sq.p, stat.p);
              stgmg::k_pack_red_sym_f64(h->st, cnt, h->tbc, dnu.back().p, dnr.back().p, dsoff.back().p,
                                        dtoff.back().p, Sq.p, D.inv64.p);
            } else {
              stgmg::k_gj_invert_f64(h->st, nb, cnt * (nblk + 1), max_n, dper, Wb.p, D.inv64.p, stat.p);
            }
            stgmg::k_fold_reduced_f64(h->st, cnt, d, D.max_nu, D.max_npr, dns.back().p, dnu.back().p, dper, nblk + 1,
                                      D.inv64.p);
          }
          HIPCHK(hipGetLastError());
        }
        HIPCHK(hipStreamSynchronize(h->st));
      } else {
        // time-block inverses: spatial MM_P, KK_P -> one (real or 2x2-block complex) matrix per
        // kept eigenvalue -> batched Gauss-Jordan, output mapped into the block layout
        const int nt = p.k + 1, nblk = h->tbc.nblk;
        const int max_ns = max_np / nt;
        bool any_c = false;
        int64_t per_patch = 0;
        std::vector<int64_t> blk_woff(nblk);
        for (int a = 0; a < nblk; ++a) {
          blk_woff[a] = per_patch;
          const int64_t na = h->tbc.cplx[a] ? 2 * max_ns : max_ns;
          per_patch += na * na;
          any_c = any_c || h->tbc.cplx[a];
        }
        const int max_n = any_c ? 2 * max_ns : max_ns;
        const int nb = stgmg::gj_panel_width(max_n, lds_limit());
        if (nb == 0) throw ApiError(STGMG_ERR_UNSUPPORTED, "patch too large for the inversion kernel");
        const int64_t sq = int64_t(max_ns) * max_ns;
        const int64_t batch =
            std::max<int64_t>(1, std::min<int64_t>(H.npatch, (int64_t(3) << 30) / ((per_patch + 2 * sq) * 8)));
        DArr<double> Wb, wmm, wkk;
        Wb.alloc(batch * per_patch, nullptr, h->st);
        wmm.alloc(batch * sq, nullptr, h->st);
        wkk.alloc(batch * sq, nullptr, h->st);
        std::vector<std::vector<stgmg::GjDesc>> descs;
        std::vector<std::vector<int32_t>> nss;
        std::vector<DArr<stgmg::GjDesc>> ddesc;
        std::vector<DArr<int32_t>> dns;
        for (int64_t p0 = 0; p0 < H.npatch; p0 += batch) {
          const int64_t cnt = std::min(batch, H.npatch - p0);
          std::vector<stgmg::GjDesc> dd(cnt * nblk);
          std::vector<int32_t> ns_of(cnt);
          for (int64_t i = 0; i < cnt; ++i) {
            const int ns = int(H.poff[p0 + i + 1] - H.poff[p0 + i]) / nt, ldh = stgmg::inv_ld(ns);
            ns_of[i] = ns;
            int64_t oo = D.ioff_h[p0 + i];
            for (int a = 0; a < nblk; ++a) {
              const bool c = h->tbc.cplx[a] != 0;
              dd[i * nblk + a] = {c ? 2 * ns : ns, ns, c ? 2 * ldh : ldh, c ? ns : 0, ldh, int32_t(p0 + i),
                                  i * per_patch + blk_woff[a], oo};
              oo += int64_t(ns) * (c ? 2 * ldh : ldh);
            }
          }
          descs.push_back(std::move(dd));
          nss.push_back(std::move(ns_of));
          ddesc.emplace_back();
          ddesc.back().upload(descs.back(), h->st, nullptr);
          dns.emplace_back();
          dns.back().upload(nss.back(), h->st, nullptr);
          stgmg::k_fill_zero(h->st, wmm.p, cnt * sq);
          stgmg::k_fill_zero(h->st, wkk.p, cnt * sq);
          stgmg::k_patch_extract_spatial_t(h->st, p0, cnt, nt, max_ns, D.poff.p, D.pdof.p, D.MMs.ptr.p, D.MMs.col.p,
                                           D.MMs.val.p, D.KKs.ptr.p, D.KKs.col.p, D.KKs.val.p, wmm.p, wkk.p);
          stgmg::k_form_time_blocks(h->st, cnt, h->tbc, max_ns, dns.back().p, wmm.p, wkk.p, ddesc.back().p, Wb.p);
          if (l == L && zero_patch >= p0 && zero_patch < p0 + cnt)
            stgmg::k_fill_zero(h->st, Wb.p + (zero_patch - p0) * per_patch + blk_woff[0],
                               (h->tbc.cplx[0] ? 4 : 1) * sq);
          if (p.smoother_prec == STGMG_FP32)
            stgmg::k_gj_invert_f32(h->st, nb, cnt * nblk, max_n, ddesc.back().p, Wb.p, D.inv32.p, stat.p);
          else
            stgmg::k_gj_invert_f64(h->st, nb, cnt * nblk, max_n, ddesc.back().p, Wb.p, D.inv64.p, stat.p);
          HIPCHK(hipGetLastError());
        }
        HIPCHK(hipStreamSynchronize(h->st));
      }
      std::vector<int32_t> st_h(H.npatch);
      HIPCHK(hipMemcpyAsync(st_h.data(), stat.p, st_h.size() * sizeof(int32_t), hipMemcpyDeviceToHost, h->st));
      HIPCHK(hipStreamSynchronize(h->st));
      for (int64_t q = 0; q < H.npatch; ++q)
        if (st_h[q])
          throw ApiError(STGMG_ERR_SINGULAR_PATCH,
                         "patch " + std::to_string(q) + " of level " + std::to_string(l) + " is singular");
      clk.lap(4);
    }
    if (l == L) {
      h->fine_info = H;
      h->fine_info.A = stgmg::Csr();
      h->fine_info.MM = stgmg::Csr();
      h->fine_info.KK = stgmg::Csr();
      h->fine_info.pdof.clear();
      h->fine_info.pdof.shrink_to_fit();
      h->fine_info.poff.clear();
      h->fine_info.tptr.clear();
      h->fine_info.tpos.clear();
      h->fine_info.winv.clear();
    }
    HIPCHK(hipStreamSynchronize(h->st));  // host vectors of H are freed below
    prev = LevelHost();
    prev.d = H.d;
    prev.r = H.r;
    prev.k = H.k;
    prev.N = H.N;
    prev.n1 = H.n1;
    prev.n1p = H.n1p;
    prev.disc = H.disc;
    prev.nlp = H.nlp;
    prev.nQ = H.nQ;
    prev.nP = H.nP;
    prev.nv = H.nv;
    prev.ns = H.ns;
    prev.n = H.n;
  }
  h->e_dev.upload(h->T.e, h->st, ctr);
  {
    std::vector<double> xq, wq, bq, bp;
    stgmg::source_tables(d, p.r, xq, wq, bq, bp, p.pressure == STGMG_PRESSURE_DISC);
    h->src_xq.upload(xq, h->st, ctr);
    h->src_wq.upload(wq, h->st, ctr);
    h->src_bq.upload(bq, h->st, ctr);
    h->src_bp.upload(bp, h->st, ctr);
    h->kfine.upload(h->fine_info.Kcell, h->st, ctr);
    HIPCHK(hipStreamSynchronize(h->st));
  }
  h->tmp_ns.alloc(h->fine_info.ns, ctr, h->st);
  h->src_buf.alloc(h->fine_info.n, ctr, h->st);
  h->xend.alloc(h->fine_info.ns, ctr, h->st);
  h->tdev.alloc(p.k + 1, ctr, h->st);
  HIPCHK(hipHostMalloc(reinterpret_cast<void**>(&h->hhost), 512 * sizeof(double), hipHostMallocDefault));
  HIPCHK(hipStreamSynchronize(h->st));
  clk.lap(0);
  if (std::getenv("STGMG_SETUP_TIMES"))
    std::fprintf(stderr,
                 "[stgmg setup] assembly and uploads %.3f s, node pairs %.3f s, coarse inverse %.3f s, transfers "
                 "%.3f s, patch solves %.3f s\n",
                 clk.sec[0], clk.sec[1], clk.sec[2], clk.sec[3], clk.sec[4]);
}

// FGMRES workspace of restart length m on n unknowns: the bases V (m+1 vectors) and Z (m), the
// Arnoldi vector w, per-block partial sums of the dot products, the Hessenberg column (two CGS
// passes and the norm) and the coefficients y of the update.
struct Krylov {
  double *V, *Z, *w, *partials, *hdev, *ydev;
};
constexpr int64_t KRYLOV_ALIGN = 32;  // doubles: every region starts 256-byte aligned
int64_t krylov_region(int64_t count) { return (count + KRYLOV_ALIGN - 1) / KRYLOV_ALIGN * KRYLOV_ALIGN; }
int64_t krylov_doubles(int64_t n, int m) {
  return krylov_region(int64_t(m + 1) * n) + krylov_region(int64_t(m) * n) + krylov_region(n) +
         krylov_region(int64_t(m + 2) * stgmg::dot_blocks(n)) + krylov_region(2 * (m + 2) + 4) + krylov_region(m + 1);
}
Krylov krylov_in(double* base, int64_t n, int m) {
  Krylov k;
  double* p = base;
  k.V = p;
  p += krylov_region(int64_t(m + 1) * n);
  k.Z = p;
  p += krylov_region(int64_t(m) * n);
  k.w = p;
  p += krylov_region(n);
  k.partials = p;
  p += krylov_region(int64_t(m + 2) * stgmg::dot_blocks(n));
  k.hdev = p;
  p += krylov_region(2 * (m + 2) + 4);
  k.ydev = p;
  return k;
}

// The handle's own workspace, allocated on first use (and grown for a longer restart).
Krylov ensure_krylov(stgmg_handle* h, int m) {
  if (h->m_alloc < m) {
    const int64_t n = h->lv[h->L].n;
    h->V.alloc(int64_t(m + 1) * n, &h->bytes, h->st);
    h->Z.alloc(int64_t(m) * n, &h->bytes, h->st);
    h->w.alloc(n, &h->bytes, h->st);
    h->partials.alloc(int64_t(m + 2) * stgmg::dot_blocks(n), &h->bytes, h->st);
    h->hdev.alloc(2 * (m + 2) + 4, &h->bytes, h->st);
    h->ydev.alloc(m + 1, &h->bytes, h->st);
    h->m_alloc = m;
  }
  return Krylov{h->V.p, h->Z.p, h->w.p, h->partials.p, h->hdev.p, h->ydev.p};
}

double device_norm2(stgmg_handle* h, const Krylov& K, const double* x, int64_t n) {
  stgmg::k_multi_dot(h->st, x, n, 1, x, n, K.partials, K.hdev, 0);
  HIPCHK(hipMemcpyAsync(h->hhost, K.hdev, sizeof(double), hipMemcpyDeviceToHost, h->st));
  HIPCHK(hipGetLastError());
  HIPCHK(hipStreamSynchronize(h->st));
  return h->hhost[0];
}

void check_solve_args(const double* rhs, const double* x, double rtol, int m, int maxit) {
  check_dev(rhs, "rhs");
  check_dev(x, "x");
  if (rhs == x) throw ApiError(STGMG_ERR_INVALID_ARG, "x must not alias rhs");
  if (m < 1 || m > 100 || maxit < 1 || !(rtol >= 0)) throw ApiError(STGMG_ERR_INVALID_ARG, "bad solver arguments");
}

// FGMRES(m) with the workspace K (the handle's own, or the static scratch of the allocation-free
// entry point); the arguments have been checked.
stgmg_status do_solve(stgmg_handle* h, const Krylov& K, const double* rhs, double* x, double rtol, int m, int maxit,
                      stgmg_info* info) {
  auto t0 = std::chrono::steady_clock::now();
  const int64_t n = h->lv[h->L].n;
  const int Lf = h->L;
  hipStream_t st = h->st;
  stgmg_info inf{};
  // r0 = rhs - A x0
  op_apply(h, Lf, 1, x, rhs, K.w);
  const double b0sq = device_norm2(h, K, K.w, n);
  if (!std::isfinite(b0sq)) throw ApiError(STGMG_ERR_NONFINITE, "non-finite initial residual (rhs or x0)");
  const double beta0 = std::sqrt(b0sq);
  inf.res0 = beta0;
  double beta = beta0;
  const double target = rtol * beta0;
  int its = 0;
  stgmg_status status = STGMG_OK;
  std::vector<double> H(size_t(m + 1) * m), cs(m), sn(m), g(m + 1), y(m);
  double est = beta0 > 0 ? 1.0 : 0.0;
  double t_vc = 0.0;
  while (beta > target && beta0 > 0) {
    if (its >= maxit) {
      status = STGMG_NOT_CONVERGED;
      break;
    }
    // v_0 = r / beta   (h->hdev[0] still holds ||r||^2 from device_norm2)
    stgmg::k_scale_copy(st, K.w, K.hdev, K.V, n);
    std::fill(H.begin(), H.end(), 0.0);
    std::fill(g.begin(), g.end(), 0.0);
    g[0] = beta;
    int jd = 0;
    for (int j = 0; j < m; ++j) {
      double* vj = K.V + int64_t(j) * n;
      double* zj = K.Z + int64_t(j) * n;
      HIPCHK(hipEventRecord(h->vc_ev[0], st));
      apply_B(h, vj, zj);
      HIPCHK(hipEventRecord(h->vc_ev[1], st));
      op_apply(h, Lf, 0, zj, nullptr, K.w);
      // classical Gram-Schmidt, twice (CGS2)
      double* h1 = K.hdev;
      double* h2 = K.hdev + (m + 2);
      double* hn = K.hdev + 2 * (m + 2);
      stgmg::k_multi_dot(st, K.V, n, j + 1, K.w, n, K.partials, h1, 0);
      stgmg::k_multi_axpy(st, K.V, n, j + 1, h1, -1.0, K.w, n);
      stgmg::k_multi_dot(st, K.V, n, j + 1, K.w, n, K.partials, h2, 0);
      stgmg::k_multi_axpy(st, K.V, n, j + 1, h2, -1.0, K.w, n);
      stgmg::k_multi_dot(st, K.w, n, 1, K.w, n, K.partials, hn, 0);
      stgmg::k_scale_copy(st, K.w, hn, K.V + int64_t(j + 1) * n, n);
      HIPCHK(hipMemcpyAsync(h->hhost, K.hdev, (2 * (m + 2) + 1) * sizeof(double), hipMemcpyDeviceToHost, st));
      HIPCHK(hipGetLastError());  // a failed launch of this iteration is reported here
      HIPCHK(hipStreamSynchronize(st));
      {
        float ms = 0.f;
        HIPCHK(hipEventElapsedTime(&ms, h->vc_ev[0], h->vc_ev[1]));
        t_vc += ms;
      }
      for (int i = 0; i <= j; ++i) H[size_t(i) * m + j] = h->hhost[i] + h->hhost[m + 2 + i];
      const double hnn = std::sqrt(h->hhost[2 * (m + 2)]);
      if (!std::isfinite(hnn)) throw ApiError(STGMG_ERR_NONFINITE, "non-finite value in the Arnoldi process");
      H[size_t(j + 1) * m + j] = hnn;
      for (int i = 0; i < j; ++i) {
        const double a = H[size_t(i) * m + j], b = H[size_t(i + 1) * m + j];
        H[size_t(i) * m + j] = cs[i] * a + sn[i] * b;
        H[size_t(i + 1) * m + j] = -sn[i] * a + cs[i] * b;
      }
      const double a = H[size_t(j) * m + j], b = H[size_t(j + 1) * m + j];
      const double den = std::hypot(a, b);
      cs[j] = den > 0 ? a / den : 1.0;
      sn[j] = den > 0 ? b / den : 0.0;
      H[size_t(j) * m + j] = den;
      H[size_t(j + 1) * m + j] = 0.0;
      g[j + 1] = -sn[j] * g[j];
      g[j] = cs[j] * g[j];
      ++its;
      jd = j + 1;
      est = std::fabs(g[j + 1]) / beta0;
      if (std::fabs(g[j + 1]) <= target || its >= maxit || hnn == 0.0) break;
    }
    // y = H^{-1} g (upper triangular), x += Z y
    for (int i = jd - 1; i >= 0; --i) {
      double s = g[i];
      for (int c = i + 1; c < jd; ++c) s -= H[size_t(i) * m + c] * y[c];
      y[i] = s / H[size_t(i) * m + i];
    }
    // through the pinned buffer (the Hessenberg reads use its first 2 (m + 2) + 1 <= 205 values)
    std::copy(y.begin(), y.begin() + jd, h->hhost + 256);
    HIPCHK(hipMemcpyAsync(K.ydev, h->hhost + 256, jd * sizeof(double), hipMemcpyHostToDevice, st));
    stgmg::k_multi_axpy(st, K.Z, n, jd, K.ydev, 1.0, x, n);
    op_apply(h, Lf, 1, x, rhs, K.w);
    beta = std::sqrt(device_norm2(h, K, K.w, n));
    if (!std::isfinite(beta)) throw ApiError(STGMG_ERR_NONFINITE, "non-finite residual");
    if (beta > target) inf.restarts++;
  }
  HIPCHK(hipGetLastError());
  HIPCHK(hipStreamSynchronize(st));
  inf.iters = its;
  inf.t_vcycle_ms = t_vc;
  inf.converged = beta <= target ? 1 : 0;
  if (!inf.converged) status = STGMG_NOT_CONVERGED;
  if (inf.converged && inf.restarts > 0) inf.restarts--;  // the final check is not a restart
  inf.rel_res_true = beta0 > 0 ? beta / beta0 : 0.0;
  inf.rel_res_est = est;
  inf.t_solve_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
  if (info) *info = inf;
  return status;
}

// Enqueue the slab right-hand side (Problem 3.1 / B.1, Def:LG) for the slab starting at t_start
// from the previous slab's end values: the source of every Radau time (from tdev[b] on the device
// when tdev is not NULL, so that a captured graph can be replayed for every slab), the jump term
// e_b MM x_prev, and their sum into rhs (rhs may be the source buffer itself).
void enqueue_slab_rhs(stgmg_handle* h, double t_start, const double* tdev, const double* x_prev_end_dev,
                      double* rhs_dev) {
  const auto& F = h->fine_info;
  const int nt = h->T.k + 1;
  for (int b = 0; b < nt; ++b) {
    stgmg::SourceArgs a{};
    a.d = F.d;
    a.r = F.r;
    a.N = F.N;
    a.nq = 1;
    for (int x = 0; x < F.d; ++x) a.nq *= F.r + 2;
    a.n1 = F.n1;
    a.n1p = F.n1p;
    a.disc = F.disc ? 1 : 0;
    a.nlp = F.nlp;
    a.nv = F.nv;
    a.ns = F.ns;
    a.h = 1.0 / F.N;
    a.rho = h->mat.rho;
    a.lam = h->mat.lambda;
    a.mu = h->mat.mu;
    a.alpha = h->mat.alpha;
    a.c0 = h->mat.c0;
    a.t = t_start + 0.5 * h->prm.tau * (1.0 + h->T.x[b]);
    a.tdev = tdev;
    a.tidx = b;
    a.scale = h->T.mt[b];
    stgmg::k_source(h->st, a, h->src_xq.p, h->src_wq.p, h->src_bq.p, h->src_bp.p, h->kfine.p,
                    h->src_buf.p + int64_t(b) * F.ns);
  }
  h->lv[h->L].MMs.apply(h->st, 0, x_prev_end_dev, nullptr, h->tmp_ns.p);
  // Problem B.1: the jump carries alpha div u^{n-1} (the volume part of C) and the boundary
  // value u_D(t_{n-1}) in place of u^{n-1} . n; MM holds all of C, so add the boundary part
  // back (u_D is zero on the boundary for the built-in solution)
  if (h->prm.form == STGMG_FORM_DTU)
    h->cface.apply(h->st, 2, x_prev_end_dev + F.nv, nullptr, h->tmp_ns.p + 2 * F.nv);
  stgmg::k_slab_rhs(h->st, nt, F.ns, h->e_dev.p, h->tmp_ns.p, h->src_buf.p, rhs_dev);
}

template <class F>
stgmg_status guarded(F&& f) {
  try {
    return f();
  } catch (const ApiError& e) {
    g_last_error = e.what();
    return e.code;
  } catch (const std::bad_alloc&) {
    g_last_error = "host out of memory";
    return STGMG_ERR_OOM;
  } catch (const std::exception& e) {
    g_last_error = e.what();
    return STGMG_ERR_HIP;
  }
}

int level_index(const stgmg_handle* h, int32_t level) {
  if (level == -1) return h->L;
  if (level < 0 || level > h->L) throw ApiError(STGMG_ERR_INVALID_ARG, "level out of range");
  return level;
}

}  // namespace

extern "C" {

stgmg_status stgmg_setup(const stgmg_params* params, void* hip_stream, stgmg_handle** out) {
  return guarded([&] {
    if (!out) throw ApiError(STGMG_ERR_INVALID_ARG, "out is NULL");
    *out = nullptr;
    check_params(params);
    std::unique_ptr<stgmg_handle> h(new stgmg_handle());
    h->prm = *params;  // K_cells is read during build() and cleared afterwards
    h->caller = reinterpret_cast<hipStream_t>(hip_stream);
    HIPCHK(hipGetDevice(&h->dev));
    if (h->dev < 0 || h->dev >= MAX_DEVICES) throw ApiError(STGMG_ERR_UNSUPPORTED, "device index out of range");
    {
      // once per device, with that device current: the device address of the static scratch
      std::lock_guard<std::mutex> lk(g_scratch_mu);
      if (!g_scratch[h->dev]) {
        void* ptr = nullptr;
        HIPCHK(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
        if (!ptr) throw ApiError(STGMG_ERR_HIP, "no device address for the static scratch");
        g_scratch[h->dev] = static_cast<double*>(ptr);
      }
    }
    HIPCHK(hipStreamCreateWithFlags(&h->own.s, hipStreamNonBlocking));
    h->st = h->own.s;
    HIPCHK(hipEventCreateWithFlags(&h->enter_ev, hipEventDisableTiming));
    HIPCHK(hipEventCreate(&h->vc_ev[0]));
    HIPCHK(hipEventCreate(&h->vc_ev[1]));
    enter(h.get());
    build(h.get());
    h->prm.K_cells = nullptr;  // copied into the level data, never kept
    for (auto& L : h->lv) L.waves = params->waves_per_patch;
    if (params->autotune) autotune(h.get());
    const int64_t nf = h->lv[h->L].n;
    // captured only on request: see the graph field of stgmg_params
    h->use_graph = params->graph == 1;
    if (h->use_graph) {
      h->gin.alloc(nf, &h->bytes, h->st);
      h->gout.alloc(nf, &h->bytes, h->st);
      capture_graph(h.get());
    }
    h->prm.K_cells = nullptr;
    *out = h.release();
    return STGMG_OK;
  });
}

stgmg_status stgmg_query(const stgmg_handle* h, int32_t level, int64_t* n_dofs, int64_t* n_patches, int64_t* nnz,
                         int64_t* hbm_bytes) {
  return guarded([&] {
    if (!h) throw ApiError(STGMG_ERR_INVALID_ARG, "NULL handle");
    const int l = level_index(h, level);
    if (n_dofs) *n_dofs = h->lv[l].n;
    if (n_patches) *n_patches = h->lv[l].npatch;
    if (nnz) *nnz = h->lv[l].MMs.nnz + h->lv[l].KKs.nnz;
    if (hbm_bytes) *hbm_bytes = h->bytes;
    return STGMG_OK;
  });
}

stgmg_status stgmg_query_launch(const stgmg_handle* h, int32_t level, int32_t* waves_per_patch,
                                int32_t* node_lanes) {
  return guarded([&] {
    if (!h) throw ApiError(STGMG_ERR_INVALID_ARG, "NULL handle");
    const int l = level_index(h, level);
    const LevelDev& L = h->lv[l];
    if (waves_per_patch) *waves_per_patch = L.sym && L.npatch > 0 ? stgmg::red_sym_waves(L.waves, L.npatch, L.max_nr) : 0;
    if (node_lanes) *node_lanes = L.node_ok ? stgmg::node_op_lanes(L.node) : 0;
    return STGMG_OK;
  });
}

stgmg_status stgmg_solve(stgmg_handle* h, const double* rhs_dev, double* x_dev, double rtol, int32_t restart,
                         int32_t max_iters, stgmg_info* info) {
  return guarded([&] {
    if (!h) throw ApiError(STGMG_ERR_INVALID_ARG, "NULL handle");
    check_solve_args(rhs_dev, x_dev, rtol, restart, max_iters);
    enter(h);
    const Krylov K = ensure_krylov(h, restart);
    return do_solve(h, K, rhs_dev, x_dev, rtol, restart, max_iters, info);
  });
}

stgmg_status stgmg_solve_noalloc(stgmg_handle* h, const double* rhs_dev, double* x_dev, double rtol,
                                 int32_t restart, int32_t max_iters, stgmg_info* info) {
  return guarded([&] {
    if (!h) throw ApiError(STGMG_ERR_INVALID_ARG, "NULL handle");
    check_solve_args(rhs_dev, x_dev, rtol, restart, max_iters);
    const int64_t n = h->lv[h->L].n;
    const int64_t need = krylov_doubles(n, restart) * int64_t(sizeof(double));
    if (need > STGMG_NOALLOC_SCRATCH_BYTES)
      throw ApiError(STGMG_ERR_UNSUPPORTED,
                     "stgmg_solve_noalloc needs " + std::to_string(need) + " bytes of workspace for " +
                         std::to_string(n) + " unknowns and restart " + std::to_string(restart) +
                         "; the static scratch holds " + std::to_string(STGMG_NOALLOC_SCRATCH_BYTES));
    double* base = g_scratch[h->dev];  // looked up by stgmg_setup on this handle's device
    if (!base) throw ApiError(STGMG_ERR_HIP, "static scratch not set up on this device");
    enter(h);
    // nothing in the workspace needs to start at zero: every region is written before it is read
    return do_solve(h, krylov_in(base, n, restart), rhs_dev, x_dev, rtol, restart, max_iters, info);
  });
}

stgmg_status stgmg_apply_operator(stgmg_handle* h, int32_t level, const double* x_dev, double* y_dev) {
  return guarded([&] {
    if (!h) throw ApiError(STGMG_ERR_INVALID_ARG, "NULL handle");
    check_dev(x_dev, "x");
    check_dev(y_dev, "y");
    enter(h);
    const int l = level_index(h, level);
    op_apply(h, l, 0, x_dev, nullptr, y_dev);
    HIPCHK(hipGetLastError());
    HIPCHK(hipStreamSynchronize(h->st));
    return STGMG_OK;
  });
}

stgmg_status stgmg_apply_vcycle(stgmg_handle* h, const double* r_dev, double* z_dev) {
  return guarded([&] {
    if (!h) throw ApiError(STGMG_ERR_INVALID_ARG, "NULL handle");
    check_dev(r_dev, "r");
    check_dev(z_dev, "z");
    enter(h);
    apply_B(h, r_dev, z_dev);
    HIPCHK(hipGetLastError());
    HIPCHK(hipStreamSynchronize(h->st));
    return STGMG_OK;
  });
}

stgmg_status stgmg_smooth(stgmg_handle* h, int32_t level, const double* b_dev, double* d_dev, int32_t sweeps) {
  return guarded([&] {
    if (!h) throw ApiError(STGMG_ERR_INVALID_ARG, "NULL handle");
    check_dev(b_dev, "b");
    check_dev(d_dev, "d");
    enter(h);
    const int l = level_index(h, level);
    if (l < 1) throw ApiError(STGMG_ERR_INVALID_ARG, "level 0 has no smoother");
    if (sweeps < 0) throw ApiError(STGMG_ERR_INVALID_ARG, "sweeps < 0");
    smooth(h, l, b_dev, d_dev, sweeps, false);
    HIPCHK(hipGetLastError());
    HIPCHK(hipStreamSynchronize(h->st));
    return STGMG_OK;
  });
}

stgmg_status stgmg_prolongate_add(stgmg_handle* h, int32_t level, const double* e_coarse_dev, double* d_fine_dev) {
  return guarded([&] {
    if (!h) throw ApiError(STGMG_ERR_INVALID_ARG, "NULL handle");
    check_dev(e_coarse_dev, "e_coarse");
    check_dev(d_fine_dev, "d_fine");
    enter(h);
    const int l = level_index(h, level);
    if (l < 1) throw ApiError(STGMG_ERR_INVALID_ARG, "level must be >= 1");
    h->lv[l].P.apply(h->st, 2, e_coarse_dev, nullptr, d_fine_dev);
    HIPCHK(hipGetLastError());
    HIPCHK(hipStreamSynchronize(h->st));
    return STGMG_OK;
  });
}

stgmg_status stgmg_restrict(stgmg_handle* h, int32_t level, const double* r_fine_dev, double* b_coarse_dev) {
  return guarded([&] {
    if (!h) throw ApiError(STGMG_ERR_INVALID_ARG, "NULL handle");
    check_dev(r_fine_dev, "r_fine");
    check_dev(b_coarse_dev, "b_coarse");
    enter(h);
    const int l = level_index(h, level);
    if (l < 1) throw ApiError(STGMG_ERR_INVALID_ARG, "level must be >= 1");
    h->lv[l].R.apply(h->st, 0, r_fine_dev, nullptr, b_coarse_dev);
    HIPCHK(hipGetLastError());
    HIPCHK(hipStreamSynchronize(h->st));
    return STGMG_OK;
  });
}

stgmg_status stgmg_slab_rhs(stgmg_handle* h, double t_start, const double* x_prev_end_dev, double* rhs_dev) {
  return guarded([&] {
    if (!h) throw ApiError(STGMG_ERR_INVALID_ARG, "NULL handle");
    check_dev(x_prev_end_dev, "x_prev_end");
    check_dev(rhs_dev, "rhs");
    enter(h);
    enqueue_slab_rhs(h, t_start, nullptr, x_prev_end_dev, rhs_dev);
    HIPCHK(hipGetLastError());
    HIPCHK(hipStreamSynchronize(h->st));
    return STGMG_OK;
  });
}

stgmg_status stgmg_march(stgmg_handle* h, double t_start, int32_t n_slabs, double* x_end_dev, double* x_dev,
                         double rtol, int32_t restart, int32_t max_iters, stgmg_info* infos) {
  return guarded([&] {
    if (!h) throw ApiError(STGMG_ERR_INVALID_ARG, "NULL handle");
    if (n_slabs < 0) throw ApiError(STGMG_ERR_INVALID_ARG, "n_slabs < 0");
    check_dev(x_end_dev, "x_end");
    check_solve_args(h->src_buf.p, x_dev, rtol, restart, max_iters);
    enter(h);
    const Krylov K = ensure_krylov(h, restart);
    const auto& F = h->fine_info;
    const int nt = h->T.k + 1;
    double* pinned_t = h->hhost + 448;  // the Radau times of one slab (the solve uses [0, 356))
    HIPCHK(hipMemcpyAsync(h->xend.p, x_end_dev, F.ns * sizeof(double), hipMemcpyDeviceToDevice, h->st));
    stgmg_status worst = STGMG_OK;
    for (int32_t sl = 0; sl < n_slabs; ++sl) {
      const double ts = t_start + double(sl) * h->prm.tau;
      if (h->rhs_exec && !h->prof) {
        // the solve of the previous slab synchronised the stream: the pinned times are free
        for (int b = 0; b < nt; ++b) pinned_t[b] = ts + 0.5 * h->prm.tau * (1.0 + h->T.x[b]);
        HIPCHK(hipMemcpyAsync(h->tdev.p, pinned_t, nt * sizeof(double), hipMemcpyHostToDevice, h->st));
        HIPCHK(hipGraphLaunch(h->rhs_exec, h->st));
      } else {
        enqueue_slab_rhs(h, ts, nullptr, h->xend.p, h->src_buf.p);
      }
      stgmg::k_fill_zero(h->st, x_dev, F.n);
      stgmg_info inf{};
      const stgmg_status st = do_solve(h, K, h->src_buf.p, x_dev, rtol, restart, max_iters, &inf);
      if (infos) infos[sl] = inf;
      if (st != STGMG_OK && worst == STGMG_OK) worst = st;
      // the end values at t_n: the last time-node block (right Radau node t_{n,k+1} = t_n)
      HIPCHK(hipMemcpyAsync(h->xend.p, x_dev + int64_t(h->T.k) * F.ns, F.ns * sizeof(double),
                            hipMemcpyDeviceToDevice, h->st));
    }
    HIPCHK(hipMemcpyAsync(x_end_dev, h->xend.p, F.ns * sizeof(double), hipMemcpyDeviceToDevice, h->st));
    HIPCHK(hipGetLastError());
    HIPCHK(hipStreamSynchronize(h->st));
    return worst;
  });
}

stgmg_status stgmg_interpolate_solution(stgmg_handle* h, double t, double* x_block_dev) {
  return guarded([&] {
    if (!h) throw ApiError(STGMG_ERR_INVALID_ARG, "NULL handle");
    check_dev(x_block_dev, "x_block");
    enter(h);
    std::vector<double> v;
    stgmg::interpolate_solution(h->fine_info, t, v);
    HIPCHK(hipMemcpyAsync(x_block_dev, v.data(), v.size() * sizeof(double), hipMemcpyHostToDevice, h->st));
    HIPCHK(hipStreamSynchronize(h->st));
    return STGMG_OK;
  });
}

stgmg_status stgmg_get_patch_inverse(stgmg_handle* h, int32_t level, int64_t patch, int32_t* n_p, double* out_host,
                                     int64_t* dofs_host) {
  return guarded([&] {
    if (!h || !n_p) throw ApiError(STGMG_ERR_INVALID_ARG, "NULL argument");
    const int l = level_index(h, level);
    if (l < 1) throw ApiError(STGMG_ERR_INVALID_ARG, "level must be >= 1");
    const LevelDev& D = h->lv[l];
    if (patch < 0 || patch >= D.npatch) throw ApiError(STGMG_ERR_INVALID_ARG, "patch out of range");
    const int n = int(D.poff_h[patch + 1] - D.poff_h[patch]);
    *n_p = n;
    if (!out_host) return STGMG_OK;
    const int64_t cnt = D.ioff_h[patch + 1] - D.ioff_h[patch];
    std::vector<double> st(cnt);
    if (h->prm.smoother_prec == STGMG_BF16) {
      std::vector<uint16_t> f(st.size());
      HIPCHK(hipMemcpyAsync(f.data(), D.inv16.p + D.ioff_h[patch], f.size() * sizeof(uint16_t), hipMemcpyDeviceToHost,
                            h->st));
      HIPCHK(hipStreamSynchronize(h->st));
      for (size_t i = 0; i < f.size(); ++i) {  // a BF16 value is the upper half of an FP32 one
        const uint32_t bits = uint32_t(f[i]) << 16;
        float v;
        std::memcpy(&v, &bits, sizeof(v));
        st[i] = v;
      }
    } else if (h->prm.smoother_prec == STGMG_FP32) {
      std::vector<float> f(st.size());
      HIPCHK(hipMemcpyAsync(f.data(), D.inv32.p + D.ioff_h[patch], f.size() * sizeof(float), hipMemcpyDeviceToHost,
                            h->st));
      HIPCHK(hipStreamSynchronize(h->st));
      for (size_t i = 0; i < f.size(); ++i) st[i] = f[i];
    } else {
      HIPCHK(hipMemcpyAsync(st.data(), D.inv64.p + D.ioff_h[patch], st.size() * sizeof(double),
                            hipMemcpyDeviceToHost, h->st));
      HIPCHK(hipStreamSynchronize(h->st));
    }
    if (!h->tb) {
      const int ld = stgmg::inv_ld(n);
      for (int a = 0; a < n; ++a)
        for (int b = 0; b < n; ++b) out_host[size_t(a) * n + b] = st[size_t(b) * ld + a];
    } else {
      // spatial block inverses X_a = (lam_a MM_P + KK_P)^{-1} (complex, ns x ns, row-major)
      const auto& tb = h->tbc;
      const int nt = tb.nt, ns = n / nt, ldh = stgmg::inv_ld(ns);
      std::vector<std::vector<std::complex<double>>> X(tb.nblk);
      if (!h->red) {
        int64_t off = 0;
        for (int a = 0; a < tb.nblk; ++a) {
          const bool c = tb.cplx[a] != 0;
          const int64_t ldc = c ? 2 * ldh : ldh;
          X[a].resize(size_t(ns) * ns);
          for (int i = 0; i < ns; ++i)
            for (int j = 0; j < ns; ++j)
              X[a][size_t(i) * ns + j] = {st[off + size_t(j) * ldc + i], c ? st[off + size_t(j) * ldc + ldh + i] : 0.0};
          off += int64_t(ns) * ldc;
        }
      } else {
        // column j of X_a: the reduced solve of the unit vector e_j
        const int d = h->prm.dim, nU = D.pnu_h[patch], nP = ns - 2 * nU, nn = nU / d, nr = nU + nP;
        const int ldn = stgmg::inv_ld(nn), ldp = stgmg::inv_ld(nP), ldr = stgmg::inv_ld(nr);
        const double* Minv = st.data();
        const double* G = Minv + size_t(nn) * ldn;  // KK_pV ((rho M)^{-1} (x) I), column-major
        int64_t off = int64_t(nn) * ldn + int64_t(nU) * ldp;
        for (int a = 0; a < tb.nblk; ++a) {
          const bool c = tb.cplx[a] != 0;
          const int64_t ldc = c ? 2 * ldr : ldr;
          const std::complex<double> lam(tb.lam[2 * a], tb.lam[2 * a + 1]);
          // S(lam)^{-1}(i, q): square column-major, or D2 X D1 from the symmetric tiles
          const std::complex<double> mu2 = std::sqrt(lam), mu1 = -1.0 / mu2;
          const int tpu = tiles_per_unit(h->prm.smoother_prec);
          const int64_t ntl = red_sym_tiles(nr, h->prm.smoother_prec);
          auto sinv = [&](int i, int q) -> std::complex<double> {
            if (!D.sym) return {st[off + size_t(q) * ldc + i], c ? st[off + size_t(q) * ldc + ldr + i] : 0.0};
            const int64_t e = stgmg::sym_slot_elem(nr, tpu, std::max(i, q), std::min(i, q));
            std::complex<double> x(st[off + e], c ? st[off + ntl * 64 + e] : 0.0);
            if (i >= nU) x *= mu2;
            if (q >= nU) x *= mu1;
            return x;
          };
          X[a].assign(size_t(ns) * ns, 0.0);
          std::vector<std::complex<double>> w(nU), z(nr), t(nr);
          for (int j = 0; j < ns; ++j) {
            std::vector<double> e(ns, 0.0);
            e[j] = 1.0;
            for (int i = 0; i < nU; ++i) {
              double acc = 0.0;
              for (int b = 0; b < nn; ++b) acc += Minv[size_t(b) * ldn + i / d] * e[b * d + i % d];
              w[i] = acc;
              z[i] = e[nU + i] + lam * e[i];
            }
            for (int x = 0; x < nP; ++x) {
              double acc = e[2 * nU + x];
              for (int q = 0; q < nU; ++q) acc += G[size_t(q) * ldp + x] * e[q];
              z[nU + x] = acc;
            }
            for (int i = 0; i < nr; ++i) {
              std::complex<double> acc = 0.0;
              for (int q = 0; q < nr; ++q) acc += sinv(i, q) * z[q];
              t[i] = acc;
            }
            for (int i = 0; i < ns; ++i)
              X[a][size_t(i) * ns + j] = i < nU ? lam * t[i] - w[i] : t[i - nU];
          }
          off += D.sym ? (c ? 2 : 1) * ntl * 64 : int64_t(nr) * ldc;
        }
      }
      // A_P^{-1}[(b,i)][(c,j)] = sum_a Q[b][a] X_a[i][j] Tin[a][c] (pairs: twice the real part)
      std::fill(out_host, out_host + size_t(n) * n, 0.0);
      for (int a = 0; a < tb.nblk; ++a) {
        const bool c = tb.cplx[a] != 0;
        for (int b = 0; b < nt; ++b)
          for (int cc = 0; cc < nt; ++cc) {
            const std::complex<double> q(tb.qout[2 * (b * tb.nblk + a)], tb.qout[2 * (b * tb.nblk + a) + 1]);
            const std::complex<double> tt(tb.tin[2 * (a * nt + cc)], tb.tin[2 * (a * nt + cc) + 1]);
            const std::complex<double> qt = q * tt;
            for (int i = 0; i < ns; ++i)
              for (int j = 0; j < ns; ++j) {
                const std::complex<double> v = qt * X[a][size_t(i) * ns + j];
                out_host[size_t(b * ns + i) * n + cc * ns + j] += c ? 2.0 * v.real() : v.real();
              }
          }
      }
    }
    if (dofs_host)
      for (int a = 0; a < n; ++a) dofs_host[a] = D.pdof_h[D.poff_h[patch] + a];
    return STGMG_OK;
  });
}

stgmg_status stgmg_footprint(const stgmg_params* params, int32_t restart, int64_t* n_dofs, int64_t* resident_bytes,
                             int64_t* setup_peak_bytes) {
  return guarded([&] {
    check_params(params);
    if (restart < 1 || restart > 100) throw ApiError(STGMG_ERR_INVALID_ARG, "restart out of range");
    const stgmg_params& p = *params;
    const int L = p.levels - 1, d = p.dim;
    const int64_t w = int64_t(value_bytes(p.smoother_prec));
    int64_t res = 0, temp_peak = 0, n_prev = 0, n_fine = 0;
    int nreal = 0, ncplx = 0;
    bool sym_ok = true;  // real kept eigenvalues > 0
    if (p.time_blocks) {
      const stgmg::TimeBlocks B = stgmg::make_time_blocks(stgmg::make_time_consts(p.k, p.tau));
      for (int a = 0; a < B.nblk; ++a) {
        (B.is_complex[a] ? ncplx : nreal)++;
        if (!B.is_complex[a] && !(B.lam[a].real() > 0.0)) sym_ok = false;
      }
    }
    for (int l = 0; l <= L; ++l) {
      const stgmg::LevelSizes S = stgmg::level_sizes(d, p.r, p.k, p.coarse_cells << l, p.patch,
                                                     p.pressure == STGMG_PRESSURE_DISC, p.form == STGMG_FORM_DTU);
      const int64_t n = S.n;
      // factored operator: spatial MM and KK; vectors b, d, r
      res += 2 * (S.ns + 1) * 8 + (S.nnzMM + S.nnzKK) * 12 + 3 * n * 8;
      {  // the velocity rows by node pairs (ptr, col, rhoM, A; cptr, ccol, C^T)
        int64_t nQ = 1;
        for (int a = 0; a < d; ++a) nQ *= int64_t(p.r) * (int64_t(p.coarse_cells) << l) + 1;
        res += 2 * (nQ + 1) * 8 + S.nodeQQ * (4 + 8 + 8 * d * d) + S.nodeQP * (4 + 8 * d);
      }
      if (l == L && p.form == STGMG_FORM_DTU) res += (S.nP + 1) * 8 + S.nnzCface * 12;  // boundary part of C
      if (l == 0) {
        res += n * stgmg::inv_ld(int(n)) * 8 + int64_t(stgmg::dense_gemv_chunks(int(n))) * n * 8;
        temp_peak = std::max(temp_peak, n * n * 8 + 3 * 32 * n * 8 + 3 * n * 8 + 64);  // W, Wb, two panels, scl, perm, src
      } else {
        res += (n + 1) * 8 + S.nnzP * 12 + (n_prev + 1) * 8 + S.nnzP * 12;
        // poff, ioff; pdof, tpos; tptr; winv; y
        res += 2 * (S.npatch + 1) * 8 + S.sum_np * 4 + S.sum_np * 4 + (n + 1) * 8 + n * 8 + S.sum_np * 8;
        if (!p.time_blocks) {
          res += (n + 1) * 8 + S.nnzA * 12;  // assembled space-time CSR for the patch extraction
          res += S.sum_np_ld * w;
          const int64_t stride = int64_t(S.max_np) * S.max_np;
          const int64_t batch =
              std::max<int64_t>(1, std::min<int64_t>(S.npatch, (int64_t(3) << 30) / (stride * 8)));
          temp_peak = std::max(temp_peak, batch * stride * 8 + batch * 8 + int64_t(sizeof(stgmg::GjDesc)) * batch +
                                              S.npatch * 4);
        } else if (p.time_blocks >= 2) {
          const int64_t max_ns = S.max_np / (p.k + 1), sq = max_ns * max_ns;
          const bool planes = red_inv_kernel(ncplx > 0, int(S.max_nr), int(S.max_nn)) != RED_INV_PANEL;
          const bool sym = red_sym_used(p, sym_ok, int(S.max_nr));
          const int64_t tiles = p.smoother_prec == STGMG_BF16   ? S.sum_tiles4
                                : p.smoother_prec == STGMG_FP32 ? S.sum_tiles2
                                                                : S.sum_tiles;
          res += (S.sum_red_fixed + (nreal + 2 * ncplx) * (sym ? tiles * 64 : S.sum_nr_ldr)) * w + S.npatch * 4;
          const int64_t per_patch = int64_t(S.max_nn) * S.max_nn +
                                    (nreal + (planes ? 2 : 4) * ncplx) * int64_t(S.max_nr) * S.max_nr;
          const int64_t sq_item = sym ? (nreal + 2 * ncplx) * int64_t(S.max_nr) * stgmg::inv_ld(S.max_nr) : 0;
          const int64_t batch = std::max<int64_t>(
              1, std::min<int64_t>(S.npatch, (int64_t(3) << 30) / ((per_patch + 2 * sq + sq_item) * 8)));
          temp_peak = std::max(temp_peak, batch * (per_patch + 2 * sq + sq_item) * 8 +
                                              2 * int64_t(sizeof(stgmg::GjDesc)) * batch * (nreal + ncplx + 1) +
                                              (sym ? 3 : 2) * batch * 4 + (sym ? 2 * batch * (nreal + ncplx) * 8 : 0) +
                                              S.npatch * 4);
        } else {
          res += (nreal + 2 * ncplx) * S.sum_ns_ldh * w;
          const int64_t max_ns = S.max_np / (p.k + 1), sq = max_ns * max_ns;
          const int64_t per_patch = (nreal + 4 * ncplx) * sq;
          const int64_t batch =
              std::max<int64_t>(1, std::min<int64_t>(S.npatch, (int64_t(3) << 30) / ((per_patch + 2 * sq) * 8)));
          temp_peak = std::max(temp_peak, batch * (per_patch + 2 * sq) * 8 +
                                              int64_t(sizeof(stgmg::GjDesc)) * batch * (nreal + ncplx) + batch * 4 +
                                              S.npatch * 4);
        }
      }
      if (l == L) {
        res += (p.k + 1) * 8 + S.ns * 8 + n * 8;  // e, MM x_prev, source
        res += S.ns * 8 + (p.k + 1) * 8;             // time marching: slab start values, Radau times
        int64_t nq = 1, nls = 1, nlp = 1, ncell = 1;
        for (int a = 0; a < d; ++a) {
          nq *= p.r + 2;
          nls *= p.r + 1;
          nlp *= p.r;
          ncell *= int64_t(p.coarse_cells) << l;
        }
        if (p.pressure == STGMG_PRESSURE_DISC) nlp = int64_t(stgmg::pdisc_exponents(p.r - 1, d).size());
        res += (4 * nq + (nls + nlp) * nq + ncell) * 8;  // device source tables and K
        const bool graph = p.graph == 1;
        if (graph) res += 2 * n * 8;
        n_fine = n;
      }
      n_prev = n;
    }
    const int64_t m = restart;
    const int64_t krylov = (2 * m + 2) * n_fine * 8 + (m + 2) * stgmg::dot_blocks(n_fine) * 8 + (2 * (m + 2) + 4) * 8 +
                           (m + 1) * 8;
    if (n_dofs) *n_dofs = n_fine;
    if (resident_bytes) *resident_bytes = res + krylov;
    if (setup_peak_bytes) *setup_peak_bytes = res + krylov + temp_peak;
    return STGMG_OK;
  });
}

stgmg_status stgmg_profile_enable(stgmg_handle* h, int32_t enable) {
  return guarded([&] {
    if (!h) throw ApiError(STGMG_ERR_INVALID_ARG, "NULL handle");
    HIPCHK(hipStreamSynchronize(h->st));
    h->prof = enable != 0;
    h->ev_used[0] = h->ev_used[1] = 0;
    return STGMG_OK;
  });
}

stgmg_status stgmg_profile_get(stgmg_handle* h, int32_t what, int64_t* launches, double* total_ms,
                               double* bytes_per_launch) {
  return guarded([&] {
    if (!h) throw ApiError(STGMG_ERR_INVALID_ARG, "NULL handle");
    if (what != STGMG_PROF_PATCH_APPLY && what != STGMG_PROF_RESIDUAL)
      throw ApiError(STGMG_ERR_INVALID_ARG, "unknown kernel class");
    HIPCHK(hipStreamSynchronize(h->st));
    double ms = 0.0;
    for (size_t i = 0; i < h->ev_used[what]; ++i) {
      float t = 0.f;
      HIPCHK(hipEventElapsedTime(&t, h->ev[what][i].first, h->ev[what][i].second));
      ms += t;
    }
    const LevelDev& F = h->lv[h->L];
    double bytes = 0.0;
    if (what == STGMG_PROF_PATCH_APPLY) {
      const double w = double(value_bytes(h->prm.smoother_prec));
      const double sum_np = F.npatch ? double(F.poff_h[F.npatch]) : 0.0;
      bytes = w * F.alg_inv_entries + 16.0 * sum_np;
    } else {
      bytes = 8.0 * F.alg_op_values + 24.0 * double(F.n);
    }
    if (launches) *launches = int64_t(h->ev_used[what]);
    if (total_ms) *total_ms = ms;
    if (bytes_per_launch) *bytes_per_launch = bytes;
    return STGMG_OK;
  });
}

stgmg_status stgmg_destroy(stgmg_handle* h) {
  return guarded([&] {
    if (h) {
      (void)hipStreamSynchronize(h->st);
      delete h;
    }
    return STGMG_OK;
  });
}

const char* stgmg_status_string(stgmg_status s) {
  switch (s) {
    case STGMG_OK: return "ok";
    case STGMG_NOT_CONVERGED: return "not converged";
    case STGMG_ERR_INVALID_ARG: return "invalid argument";
    case STGMG_ERR_UNSUPPORTED: return "unsupported configuration";
    case STGMG_ERR_OOM: return "out of memory";
    case STGMG_ERR_HIP: return "HIP error";
    case STGMG_ERR_SINGULAR_PATCH: return "singular patch matrix";
    case STGMG_ERR_NONFINITE: return "non-finite value";
    case STGMG_ERR_BAD_POINTER: return "bad device pointer";
    case STGMG_PENDING: return "pending";
    default: return "unknown status";
  }
}

const char* stgmg_last_error(void) { return g_last_error.c_str(); }

}  // extern "C"
