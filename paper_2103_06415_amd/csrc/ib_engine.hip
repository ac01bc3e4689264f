// Host engine and C-ABI of the immersed-boundary solver (see include/ibfsi.h).
//
// A step (Sec. 2.3 and 3.3; Algorithm 2) is enqueued on the solver's stream as:
//   for every level, coarse to fine:
//     ring of the level from the coarser level's new streamfunction
//     explicit right-hand side + row DST       (k_rhs_rowdst)
//     column DST, spectral solve, inverse      (k_col_solve)
//     inverse row DST -> new streamfunction   (k_row_idst)   [level 0: only the rows
//                                                             the bodies need -> s*]
//   level 0 with bodies: FSI iterations (body operator, Schur matrix, LU, structure
//   update; the host reads the convergence measure), then the corrector source, its
//   row DST, the column solve accumulated into level 0's spectral rows, and the final
//   inverse row DST.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <atomic>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstring>
#include <functional>
#include <list>
#include <map>
#include <memory>
#include <mutex>
#include <shared_mutex>
#include <string>
#include <vector>

#include "ib_body.hpp"
#include "ib_internal.hpp"
#include "ibfsi.h"

using namespace ib;

namespace {

// refinement sweeps launched per Schur solve; one that has not converged by then makes
// the solver rebuild its approximate inverse
constexpr int REFINE_MAXIT = 16;
// Refresh policy of the approximate Schur inverse in the automatic mode: one Newton-Schulz
// step at every FSI iteration up to this many stress unknowns (the two n^3 products cost
// less than the refinement sweeps they save); above it, only at the first iteration of a
// step whose previous stress solve needed more than REFRESH_SWEEPS sweeps.
constexpr int REFRESH_ALL_NF = 256;
constexpr int REFRESH_SWEEPS = 6;

// ---- offline operator cache
// The offline stage's product depends only on the grid, dt, Re and the sub-domain (plus
// the points of stationary bodies): B' for moving bodies (Algorithm 1), the unscaled
// Schur matrix G = E C (C^T A C)^{-1} C^T E^T for stationary ones.  A process-wide host
// cache keyed by exactly those numbers lets later solvers (e.g. the requests of a
// parametric study) skip the offline stage; entries are shared read-only, evicted least
// recently used beyond a byte limit, and a solver that finds its key being built by
// another thread waits for it.  ib_export_operator / ib_import_operator move the same
// data across processes.
struct OpData {
  std::vector<double> key;
  std::vector<int64_t> ptr;  // B': CSR rows (empty for G)
  std::vector<int32_t> col;
  std::vector<double> val;   // B' values, or G row-major with pitch pm
  size_t bytes() const { return ptr.size() * 8 + col.size() * 4 + val.size() * 8 + key.size() * 8; }
};
using OpPtr = std::shared_ptr<const OpData>;

struct OpCache {
  std::mutex mu;
  std::condition_variable cv;
  std::list<OpPtr> lru;                 // most recent first
  std::vector<std::vector<double>> building;
  size_t bytes = 0;
  size_t limit = (size_t)8 << 30;
};
OpCache& op_cache() {
  static OpCache c;
  return c;
}

// Find key; if another thread is building it, wait.  Returns null when absent (and then
// registers the caller as its builder, who must then call op_cache_done).
OpPtr op_cache_get(const std::vector<double>& key) {
  OpCache& c = op_cache();
  std::unique_lock<std::mutex> lk(c.mu);
  if (c.limit == 0) return nullptr;
  for (;;) {
    for (auto it = c.lru.begin(); it != c.lru.end(); ++it)
      if ((*it)->key == key) {
        OpPtr p = *it;
        c.lru.erase(it);
        c.lru.push_front(p);
        return p;
      }
    if (std::find(c.building.begin(), c.building.end(), key) == c.building.end()) {
      c.building.push_back(key);
      return nullptr;
    }
    c.cv.wait(lk);
  }
}

void op_cache_done(const std::vector<double>& key, OpPtr p) {
  OpCache& c = op_cache();
  std::lock_guard<std::mutex> lk(c.mu);
  auto b = std::find(c.building.begin(), c.building.end(), key);
  if (b != c.building.end()) c.building.erase(b);
  if (p && c.limit > 0 && p->bytes() <= c.limit) {
    c.lru.push_front(p);
    c.bytes += p->bytes();
    while (c.bytes > c.limit && !c.lru.empty()) {
      c.bytes -= c.lru.back()->bytes();
      c.lru.pop_back();
    }
  }
  c.cv.notify_all();
}

struct HostBody {
  int kind = BODY_RIGID;
  int m = 0;
  double ds = 0;
  std::vector<double> xy, ub;                       // rigid
  double hx = 0, hy = 0, length = 0, theta0 = 0, inertia = 0, stiffness = 0, damping = 0;
  double theta = 0, phi = 0;                        // torsional
  std::vector<double> xy_ref, xy0, rot0;            // deformable
  double mass = 0, ei = 0, ea = 0;
  ib_motion_fn motion = nullptr;                    // moving rigid: pose callback
  void* motion_ctx = nullptr;
  double pose[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};     // its pose, rates, accelerations (last step)
  int driver = -1;                                  // torsional on a driver: its body index
  double hbx = 0, hby = 0, theta_rel = 0, cg = 0;   //   hinge in the driver's frame, angles
};

// Frame of a mounted torsional body (MOUNT_W doubles, layout in ib_body.hpp) from its
// driver's pose, rates and accelerations q[9] at the same time.
void mount_frame(const HostBody& mb, const double* q, double* out) {
  const double c = std::cos(q[2]), sn = std::sin(q[2]);
  const double rx = c * mb.hbx - sn * mb.hby, ry = sn * mb.hbx + c * mb.hby;
  out[MF_HX] = q[0] + rx;
  out[MF_HY] = q[1] + ry;
  out[MF_ANG] = q[2] + mb.theta_rel;
  out[MF_VX] = q[3] - q[5] * ry;
  out[MF_VY] = q[4] + q[5] * rx;
  out[MF_OM] = q[5];
  out[MF_AX] = q[6] - q[8] * ry - q[5] * q[5] * rx;
  out[MF_AY] = q[7] + q[8] * rx - q[5] * q[5] * ry;
  out[MF_AL] = q[8];
  out[MOUNT_W - 1] = 0.0;
}

// Its pseudo-moment at deflection th (the device's tors_g, for the initial state).
double mount_g(const HostBody& mb, const double* fr, double th) {
  const double ph = fr[MF_ANG] + th;
  return -mb.inertia * fr[MF_AL] - mb.mass * mb.cg * (std::cos(ph) * fr[MF_AY] - std::sin(ph) * fr[MF_AX]);
}

struct LevelState {
  double h = 0, alpha = 0;
  void* s = nullptr;     // streamfunction, (n+1) rows with the ring
  void* g = nullptr;     // circulation C^T C s at interior vertices, (n-1) rows
  void* hist = nullptr;
  void* sring = nullptr;
  void* gring[2] = {nullptr, nullptr};
  int gcur = 0;
};

inline int round_up(int v, int m) { return (v + m - 1) / m * m; }

}  // namespace

struct Offline {
  int nslots = 0;
  double* srcrows = nullptr;  // [nslots][6][pitch]
  int* rfirst = nullptr;
  double* X = nullptr;        // [nslots][(n-1) pitch]
  double* S = nullptr;        // [nslots][(n+1) pitch]
  double* vals = nullptr;     // [nslots][ntarget]
};

// Configurations of the single-precision transform kernels chosen for one grid size, with
// the measured average launch times (microseconds; 0 = not measured).
struct FlowTuning {
  int n = 0;
  int rhs = 0, col = 0, idst = 0;
  double rhs_us[ib::FLOW_VARIANTS] = {}, col_us[ib::FLOW_VARIANTS] = {},
         idst_us[ib::FLOW_VARIANTS] = {};
};

// Recording a graph and the library's other HIP calls exclude each other across threads:
// while a stream records, this runtime rejects synchronising calls (and synchronous copies
// on the legacy stream) from every thread.  Entry points that call HIP hold the shared
// side; recording takes the exclusive side when it is free.  (HIP calls that the application makes
// itself on other threads while a solver records are not covered.)
static std::shared_mutex g_hip_mu;
std::shared_lock<std::shared_mutex> ib::hip_shared_lock() {
  return std::shared_lock<std::shared_mutex>(g_hip_mu);
}
struct HipShared {
  std::shared_lock<std::shared_mutex> l{g_hip_mu};
};

// Solvers of the process inside ib_step right now.  The next step's levels are launched
// early (side stream or during the host wait) only while a solver steps alone: several
// solvers stepping at once already fill the GPU, and the extra stream's event waits then
// hold up the other solvers' work on the runtime's few hardware queues.
static std::atomic<int> g_stepping{0};

// A recorded step: its executable graph and the number of FSI iterations it launches ahead.
struct StepGraph {
  hipGraphExec_t exec = nullptr;
  int K = 0;
  bool refresh0 = false;
};

struct ib_solver {
  ib_config cfg{};
  ib_allocator alloc{};
  bool has_alloc = false;
  hipStream_t stream = nullptr;
  int n = 0, pitch = 0;
  int ny = 0;          // cells along y (n on a square level)
  void* twy = nullptr;   // rectangular levels: transform tables of length ny, in the flow
  void* lamy = nullptr;  //   precision, and sin(pi k / n), k <= n (the x axis)
  void* sinx = nullptr;
  bool fp64 = true;
  bool gemm = false;  // predictor transforms as BF16-split products on the matrix cores
  FlowTuning tune;    // kernel configurations of the row and column transforms
  bool tune_forced = false;
  int kpad = 0;       // size of the padded sine matrix
  int gemm_tn = 0;    // measured stage depth in k of the sine-transform products (64 or 128)
  void* shi = nullptr;
  void* slo = nullptr;
  float* sinv = nullptr;
  float* ys = nullptr;
  float* yg = nullptr;
  size_t es = 8;
  std::vector<LevelState> lv;
  void* work = nullptr;   // spectral rows of s (then s-transform rows)
  void* workg = nullptr;  // the same for the circulation
  void* work2 = nullptr;
  void* work_pre = nullptr;   // spectral scratch of the levels launched ahead
  void* workg_pre = nullptr;
  void* lift_pre = nullptr;   // edge transforms of the rings of the levels launched ahead
  void* lift_l1 = nullptr;    // edge transforms of level 1's next ring, made on `side`
  bool top_ahead = false;     // the next step's coarsest level is already on the stream
  int ahead_mode = 2;         // IB_OPT_TOP_AHEAD: 0 off, 1 coarsest level, 2 side stream
  hipEvent_t ctl_ready = nullptr;  // this step's control block is on the host
  hipStream_t side = nullptr;      // the next step's levels >= 2 (ahead_mode 2)
  hipEvent_t l1_done = nullptr;    // level 1's state of this step is final (on `stream`)
  hipEvent_t side_done = nullptr;  // the levels launched on `side` are done
  bool side_ahead = false;         // this step's levels >= 2 were launched on `side`
  bool ctl_early = false;          // copy the control block right after the FSI iterations
  void* lift = nullptr;   // edge transforms of a new streamfunction ring, [4][n-1]
  void* sstar = nullptr;
  void* tw = nullptr;
  void* lam = nullptr;
  void* tw64 = nullptr;
  void* lam64 = nullptr;
  std::vector<std::vector<double>> omega0;
  std::vector<HostBody> bodies;
  bool has_sd = false;
  std::vector<std::array<double, 4>> sd_rects;  // sub-domain rectangles (x0, x1, y0, y1)
  bool prepared = false, failed = false, first = true;
  bool allocated = false;  // level state lives on the device (from ib_prepare on)
  bool released = false;   // device memory given back; results kept on the host
  std::vector<double> h_f, h_tors, h_chi, h_vort0;
  // Schur solves without the device-wide barrier: LU of a copy of M (lu_always when the
  // refinement's workgroups cannot all be resident; lu_step for the rest of a step whose
  // refinement barrier timed out); barrier_spin: the barrier's spin bound (0: default)
  bool lu_always = false, lu_step = false;
  int64_t solve_fallbacks = 0;
  long barrier_spin = 0;       // as set by IB_OPT_BARRIER_SPIN
  bool barrier_force = false;  // IB_OPT_BARRIER_FORCE_TIMEOUT
  // the refinement kernels' barrier argument: the bound, negated when every wait must time out
  long barrier_arg() const {
    const long b = barrier_spin > 0 ? barrier_spin : (1L << 22);
    return barrier_force ? -b : barrier_spin;
  }
  // no-slip residual and body forces of the last step (k_outputs), for step out_step
  double* dout = nullptr;
  std::vector<double> h_out;
  int64_t out_step = -1;
  int64_t step = 0;
  int iters_last = 0, iters_max = 0;
  double delta_last = 0;
  double prepare_seconds = 0;
  std::vector<std::pair<void*, size_t>> allocs;
  std::string last_error;

  // ---- bodies on the device
  int npts = 0, nf = 0, ntors = 0, ndef = 0, ndof = 0, nel_total = 0;
  bool use_sd = false, stationary = false;
  ib::SdBoxes sdb{};          // the rectangles snapped to level-0 vertices
  int sd_ilo = 0, sd_ihi = 0, sd_jlo = 0, sd_jhi = 0;  // vertex bounds of their union
  int sd_ngrid = 0, sd_total = 0;
  int64_t bp_nnz = 0;
  // exact operator for moving bodies: G = E C (C^T A C)^{-1} C^T E^T rebuilt at every FSI
  // iterate from point-source columns (no sub-domain)
  bool exact_moving = false;
  Offline xo;
  OffRows xrows{};
  double* gx = nullptr;
  std::shared_ptr<const OpData> op;        // offline operator in use (built, cached or imported)
  std::shared_ptr<const OpData> imported;  // from ib_import_operator, checked at prepare
  int op_source = 0;                       // 0 built, 1 from the cache, 2 imported
  int blo = 1, bhi = 1, bilo = 1, bihi = 1;  // rows / columns the bodies can touch
  FsiArgs fa{};
  double* f = nullptr;
  double* rhs = nullptr;
  double* Minv = nullptr;   // stationary: exact inverse; moving: approximate inverse X
  double* Xn = nullptr;     // Newton-Schulz workspace
  double* W = nullptr;
  double* Mtmp = nullptr;
  double* rinfo = nullptr;  // refinement workspace (device)
  bool x_valid = false;
  bool x_valid_retry = false;
  int* gate = nullptr;      // device gates of the FSI iterations launched ahead (in ctl)
  bool fsi_ahead = true;    // launch a step's FSI iterations ahead of their tests
  int nmov = 0;             // rigid bodies in prescribed motion
  int nmount = 0;           // torsional bodies mounted on them
  double* hpose = nullptr;  // pinned staging of their poses, two sets (alternate steps)
  bool graphs = false;      // replay recorded steps as HIP graphs
  int refresh_mode = 2;     // Newton-Schulz refresh of X: IB_OPT_REFRESH_EVERY_ITER's value
  static constexpr int GRAPH_SLOTS = 4;
  StepGraph step_graphs[2][GRAPH_SLOTS];  // by ring-buffer alternation, then by K
  int graph_next[2] = {0, 0};             // slot to reuse next (round robin)
  int64_t graph_captures = 0, graph_launches = 0, fsi_resumes = 0, graph_failures = 0;
  int inverse_rebuilds = 0;
  // sweeps launched per stress solve in tolerance mode, per FSI iteration index (0, 1, 2, 3+)
  // control block read back once per FSI iteration: error flags (2 ints), max |delta|,
  // refinement residual and sweeps; one device copy and its pinned host mirror
  void* ctl = nullptr;
  void* hctl = nullptr;
  int* flags = nullptr;
  double* delta = nullptr;
  double* rout = nullptr;
  int* hflags = nullptr;
  double* hdelta = nullptr;
  double* hrinfo = nullptr;
  std::vector<double> ds_rows;
  // kernel timing
  bool timing = false;
  struct Ev { hipEvent_t a, b; int cls; };
  std::vector<Ev> events;
  std::vector<hipEvent_t> event_pool;
  int64_t t_count[IB_K_CLASSES] = {0};
  double t_ms[IB_K_CLASSES] = {0};
};

// Fixed device scratch of the allocation-free entry point (ib_op_solve_noalloc): one copy
// per GPU, reached from host code only through its address from hipGetSymbolAddress.
constexpr size_t kNoallocScratchBytes = 64 * 1024;
constexpr int kMaxDevices = 64;
static __device__ __align__(256) unsigned char scratch[kNoallocScratchBytes];

namespace {

ib_status hip_fail(ib_solver* s, hipError_t e, const char* what) {
  if (s) s->last_error = std::string(what) + ": " + hipGetErrorString(e);
  return IB_ERR_HIP;
}

#define HIPCHK(expr)                                   \
  do {                                                 \
    hipError_t e_ = (expr);                            \
    if (e_ != hipSuccess) return hip_fail(s, e_, #expr); \
  } while (0)

// The same check for code that has no solver handle.
#define HIPRET(expr)                                 \
  do {                                               \
    if ((expr) != hipSuccess) return IB_ERR_HIP;     \
  } while (0)

void* dalloc(ib_solver* s, size_t bytes) {
  if (bytes == 0) bytes = 8;
  void* p = nullptr;
  if (s->has_alloc) {
    p = s->alloc.alloc(bytes, s->alloc.ctx);
  } else if (hipMalloc(&p, bytes) != hipSuccess) {
    p = nullptr;
  }
  if (p) s->allocs.push_back({p, bytes});
  return p;
}

void dfree(ib_solver* s, void* p) {
  if (!p) return;
  for (size_t k = 0; k < s->allocs.size(); ++k)
    if (s->allocs[k].first == p) {
      s->allocs.erase(s->allocs.begin() + k);
      break;
    }
  if (s->has_alloc) s->alloc.free(p, s->alloc.ctx);
  else (void)hipFree(p);
}

// Twiddles exp(-i pi m / n), m < 2n, and 1-D eigenvalues 4 sin^2(pi k / 2n), k < n.
// Transform tables of grid size n: twiddles exp(-i pi m / n), m < 2n, as (re, im) pairs in
// t[0 .. 4n), and the 1-D eigenvalues 4 sin^2(pi k / 2n), k = 1 .. n-1, in l[0 .. n-1).
template <typename T>
void table_values(int n, T* t, T* l) {
  for (int m = 0; m < 2 * n; ++m) {
    const long double a = 3.14159265358979323846264338327950288L * (long double)m / (long double)n;
    t[2 * m] = (T)std::cos((double)a);
    t[2 * m + 1] = (T)-std::sin((double)a);
  }
  for (int k = 1; k < n; ++k) {
    const double v = std::sin(M_PI * k / (2.0 * n));
    l[k - 1] = (T)(4.0 * v * v);
  }
}

template <typename T>
ib_status make_tables(ib_solver* s, int n, void** tw, void** lam) {
  std::vector<T> t(4 * n), l(n);
  table_values<T>(n, t.data(), l.data());
  *tw = dalloc(s, t.size() * sizeof(T));
  *lam = dalloc(s, l.size() * sizeof(T));
  if (!*tw || !*lam) return IB_ERR_OOM;
  HIPCHK(hipMemcpy(*tw, t.data(), t.size() * sizeof(T), hipMemcpyHostToDevice));
  HIPCHK(hipMemcpy(*lam, l.data(), l.size() * sizeof(T), hipMemcpyHostToDevice));
  return IB_OK;
}

// Rectangular levels: the y axis's transform tables (length ny) and sin(pi k / nx), k <= nx,
// which the column solve needs for the x transforms of the ring's bottom and top edges.
template <typename T>
ib_status make_rect_tables(ib_solver* s) {
  ib_status st = make_tables<T>(s, s->ny, &s->twy, &s->lamy);
  if (st) return st;
  std::vector<T> sx(s->n + 1);
  for (int k = 0; k <= s->n; ++k) sx[k] = (T)std::sin(M_PI * k / s->n);
  s->sinx = dalloc(s, sx.size() * sizeof(T));
  if (!s->sinx) return IB_ERR_OOM;
  HIPCHK(hipMemcpy(s->sinx, sx.data(), sx.size() * sizeof(T), hipMemcpyHostToDevice));
  return IB_OK;
}

// The operator solve of ib_op_solve on its tables: row transform of `in` into `out`, column
// transform, spectral divide and inverse, inverse row transform, all in `out`.
template <typename T>
ib_status op_solve_run(int n, int pitch, hipStream_t st, double alpha, const void* in, void* out,
                       const void* tw, const void* lam) {
  RowArgs<T> r{};
  r.in = static_cast<const T*>(in);
  r.out = static_cast<T*>(out);
  r.pi = r.po = pitch;
  r.r0 = 1;
  r.r1 = n - 1;
  HIPRET(launch_rowdst<T>(r, n, 1, tw, st));
  ColArgs<T> c{};
  c.in = static_cast<T*>(out);
  c.out = static_cast<T*>(out);
  c.pi = c.po = pitch;
  c.r0 = 1;
  c.r1 = n - 1;
  c.alpha = (T)alpha;
  c.scale = (T)(4.0 / ((double)n * n));
  c.w0 = 1;
  c.w1 = n - 1;
  HIPRET(launch_col_solve<T>(c, n, 1, tw, lam, st));
  r.in = static_cast<const T*>(out);
  r.interior_out = 1;
  HIPRET(launch_row_idst<T>(r, n, 1, tw, nullptr, 0, st));
  return IB_OK;
}

// ---- fixed device scratch of the allocation-free entry point ----
// ib_op_solve_noalloc keeps the transform tables that ib_op_solve allocates per call in this
// file-scope device array instead.  Each GPU the library runs on holds its own copy, at its
// own address, until the process ends.  In host code the array's name is only a stand-in:
// its device address comes from hipGetSymbolAddress, once per device, and only that address
// is handed to kernels and copies.
static std::mutex g_scratch_mu;
static void* g_scratch_ptr[kMaxDevices] = {};

// Device address of `scratch` on the current device (looked up at the first call there).
static ib_status scratch_address(void** out) {
  int dev = 0;
  HIPRET(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices) return IB_ERR_HIP;
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || p == nullptr) return IB_ERR_HIP;
    g_scratch_ptr[dev] = p;
  }
  *out = g_scratch_ptr[dev];
  return IB_OK;
}

// Bytes of scratch the tables of size n take: twiddles (4n values) from offset 0, eigenvalues
// (n - 1 values) from the next 256-byte boundary.
template <typename T>
size_t noalloc_lam_offset(int n) {
  return ((size_t)4 * n * sizeof(T) + 255) / 256 * 256;
}
template <typename T>
size_t noalloc_bytes(int n) {
  return noalloc_lam_offset<T>(n) + (size_t)n * sizeof(T);
}

template <typename T>
ib_status op_solve_noalloc_run(int n, int pitch, hipStream_t st, double alpha, const void* in,
                               void* out) {
  if (noalloc_bytes<T>(n) > kNoallocScratchBytes) return IB_ERR_SCRATCH;
  void* base = nullptr;
  ib_status rc = scratch_address(&base);
  if (rc) return rc;
  // host tables in a fixed buffer (no heap): 4n + n values; larger sizes are refused
  constexpr int kMaxN = 1280;
  if (n > kMaxN) return IB_ERR_SCRATCH;
  T host[5 * kMaxN];
  T* ht = host;
  T* hl = host + 4 * n;
  table_values<T>(n, ht, hl);
  unsigned char* b = static_cast<unsigned char*>(base);
  void* tw = b;
  void* lam = b + noalloc_lam_offset<T>(n);
  if (hipMemcpyAsync(tw, ht, (size_t)4 * n * sizeof(T), hipMemcpyHostToDevice, st) != hipSuccess ||
      hipMemcpyAsync(lam, hl, (size_t)(n - 1) * sizeof(T), hipMemcpyHostToDevice, st) != hipSuccess)
    rc = IB_ERR_HIP;
  if (!rc) rc = op_solve_run<T>(n, pitch, st, alpha, in, out, tw, lam);
  // on every path the host tables outlive their copies; the solve is complete on return, as
  // for ib_op_solve
  const hipError_t e = hipStreamSynchronize(st);
  if (rc) return rc;
  return e == hipSuccess ? IB_OK : IB_ERR_HIP;
}

// ------------------------------------------------------------- flow helpers

template <typename T>
ib_status solve_into(ib_solver* s, void* work, double alpha, double scale, int r0, int r1,
                     const void* tw, const void* lam, void* workg = nullptr,
                     const void* lift = nullptr, int var = 0, hipEvent_t ev0 = nullptr,
                     hipEvent_t ev1 = nullptr) {
  ColArgs<T> c{};
  c.ev0 = ev0;
  c.ev1 = ev1;
  c.var = var;
  c.in = static_cast<T*>(work);
  c.out = static_cast<T*>(work);
  c.out2 = static_cast<T*>(workg);
  c.lift = static_cast<const T*>(lift);
  c.pi = c.po = s->pitch;
  c.r0 = r0;
  c.r1 = r1;
  c.alpha = (T)alpha;
  c.scale = (T)scale;
  c.w0 = 1;
  c.w1 = s->ny - 1;
  if (s->ny != s->n) {
    // rectangular level: the column transform runs along y with the y tables; the x
    // eigenvalues and sines come with the columns
    c.ncols = s->n - 1;
    c.lamx = static_cast<const T*>(lam);
    c.sinx = static_cast<const T*>(s->sinx);
    HIPCHK(launch_col_solve<T>(c, s->ny, 1, s->twy, s->lamy, s->stream));
    return IB_OK;
  }
  HIPCHK(launch_col_solve<T>(c, s->n, 1, tw, lam, s->stream));
  return IB_OK;
}

// Transform tables of the y axis (the x axis's on a square level).
inline const void* twy_of(const ib_solver* s) { return s->ny != s->n ? s->twy : s->tw; }

// Initial streamfunction of every level from its vorticity, coarse to fine.
template <typename T>
ib_status init_streamfunction(ib_solver* s) {
  const int n = s->n, ny = s->ny, G = (int)s->lv.size(), P = s->pitch;
  std::vector<T> host((size_t)(ny - 1) * P, T(0));
  for (int g = G - 1; g >= 0; --g) {
    LevelState& L = s->lv[g];
    if (g < G - 1) {
      HIPCHK(launch_ring<T>(static_cast<T*>(s->lv[g + 1].s), P, static_cast<T*>(s->lv[g + 1].g), P,
                            n, ny, static_cast<T*>(L.sring), static_cast<T*>(L.gring[L.gcur]),
                            s->stream));
    }
    std::fill(host.begin(), host.end(), T(0));
    if (g < (int)s->omega0.size() && !s->omega0[g].empty()) {
      const double h2 = L.h * L.h;
      for (int j = 0; j < ny - 1; ++j)
        for (int i = 0; i < n - 1; ++i)
          host[(size_t)j * P + i] = (T)(h2 * s->omega0[g][(size_t)j * (n - 1) + i]);
    }
    HIPCHK(hipMemcpyAsync(s->work, host.data(), host.size() * sizeof(T), hipMemcpyHostToDevice,
                          s->stream));
    HIPCHK(hipMemcpyAsync(L.g, host.data(), host.size() * sizeof(T), hipMemcpyHostToDevice,
                          s->stream));
    if (g < G - 1)
      HIPCHK(launch_ring_edge_dst<T>(static_cast<T*>(L.sring), n, ny, s->tw, twy_of(s),
                                     static_cast<T*>(s->lift), s->stream));
    RowArgs<T> r{};
    r.in = static_cast<T*>(s->work);
    r.out = static_cast<T*>(s->work);
    r.pi = r.po = P;
    r.r0 = 1;
    r.r1 = ny - 1;
    r.ny = ny;
    HIPCHK(launch_rowdst<T>(r, n, 1, s->tw, s->stream));
    ib_status st = solve_into<T>(s, s->work, 0.0, 4.0 / ((double)n * ny), 1, ny - 1, s->tw, s->lam,
                                 nullptr, g < G - 1 ? s->lift : nullptr);
    if (st) return st;
    RowArgs<T> q = r;
    q.out = static_cast<T*>(L.s);
    HIPCHK(launch_row_idst<T>(q, n, 1, s->tw, g < G - 1 ? static_cast<T*>(L.sring) : nullptr, 1,
                              s->stream));
    HIPCHK(hipStreamSynchronize(s->stream));  // host buffer is reused
  }
  return IB_OK;
}

// ---------------------------------------------------------------- offline

// Batched columns of E C K C^T E^T (K = [L (I + alpha L)]^{-1}) for the rows of
// `src` sampled at the rows of `dst`: vals[b * ntarget + t] for b < nslots.

ib_status offline_columns(ib_solver* s, Offline& w, const OffRows& src, int col0, int ncols,
                          const OffRows& dst, int ntarget, int tlo, int thi) {
  const int n = s->n, P = s->pitch;
  const int ns = std::min(w.nslots, ncols - col0);
  const double alpha = s->lv[0].alpha;
  HIPCHK(launch_point_source_rowdst(src, col0, ncols, ns, s->tw64, w.srcrows, P, (size_t)6 * P,
                                    w.rfirst, s->stream));
  ColArgs<double> c{};
  c.in = w.srcrows;
  c.out = w.X;
  c.pi = c.po = P;
  c.r0 = 1;
  c.r1 = n - 1;
  c.alpha = alpha;
  c.scale = 4.0 / ((double)n * n);
  c.bsi = (size_t)6 * P;
  c.bso = (size_t)(n - 1) * P;
  c.rfirst = w.rfirst;
  c.rcount = 6;
  c.w0 = tlo;
  c.w1 = thi;
  HIPCHK(launch_col_solve<double>(c, n, ns, s->tw64, s->lam64, s->stream));
  RowArgs<double> r{};
  r.in = w.X;
  r.out = w.S;
  r.pi = r.po = P;
  r.r0 = tlo;
  r.r1 = thi;
  r.bsi = (size_t)(n - 1) * P;
  r.bso = (size_t)(n + 1) * P;
  HIPCHK(launch_row_idst<double>(r, n, ns, s->tw64, nullptr, 0, s->stream));
  HIPCHK(launch_sample(dst, ntarget, w.S, P, (size_t)(n + 1) * P, w.vals, ns, s->stream));
  return IB_OK;
}

ib_status offline_alloc(ib_solver* s, Offline& w, int nslots, int ntarget) {
  const int n = s->n, P = s->pitch;
  w.nslots = nslots;
  w.srcrows = static_cast<double*>(dalloc(s, (size_t)nslots * 6 * P * 8));
  w.rfirst = static_cast<int*>(dalloc(s, (size_t)nslots * 4));
  w.X = static_cast<double*>(dalloc(s, (size_t)nslots * (n - 1) * P * 8));
  w.S = static_cast<double*>(dalloc(s, (size_t)nslots * (n + 1) * P * 8));
  w.vals = static_cast<double*>(dalloc(s, (size_t)nslots * ntarget * 8));
  if (!w.srcrows || !w.rfirst || !w.X || !w.S || !w.vals) return IB_ERR_OOM;
  HIPCHK(hipMemsetAsync(w.S, 0, (size_t)nslots * (n + 1) * P * 8, s->stream));
  return IB_OK;
}

void offline_free(ib_solver* s, Offline& w) {
  dfree(s, w.srcrows);
  dfree(s, w.rfirst);
  dfree(s, w.X);
  dfree(s, w.S);
  dfree(s, w.vals);
  w = Offline{};
}

int offline_slots(ib_solver* s, int ntarget) {
  // keep the batch buffers near 1 GiB
  const size_t per = (size_t)(2 * s->n + 6) * s->pitch * 8 + (size_t)ntarget * 8;
  size_t k = ((size_t)1 << 30) / per;
  if (k > 256) k = 256;
  if (k < 1) k = 1;
  return (int)k;
}

// Bracket the enclosed launches with events when timing is enabled.
struct TimeScope {
  ib_solver* s;
  int cls;
  hipEvent_t b = nullptr;
  hipEvent_t e = nullptr;
  hipEvent_t take() {
    if (!s->event_pool.empty()) {
      hipEvent_t v = s->event_pool.back();
      s->event_pool.pop_back();
      return v;
    }
    hipEvent_t v = nullptr;
    (void)hipEventCreate(&v);
    return v;
  }
  bool ext = false;  // the scope's one launch records b and e itself (hipExtLaunchKernelGGL)
  TimeScope(ib_solver* s_, int c, bool ext_ = false) : s(s_), cls(c), ext(ext_) {
    if (!s->timing) return;
    b = take();
    e = take();
    if (!ext) (void)hipEventRecord(b, s->stream);
  }
  ~TimeScope() {
    if (!s->timing || !b) return;
    if (!ext) (void)hipEventRecord(e, s->stream);
    s->events.push_back({b, e, cls});
  }
};

void harvest_events(ib_solver* s) {
  (void)hipStreamSynchronize(s->stream);
  for (auto& ev : s->events) {
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, ev.a, ev.b) == hipSuccess) {
      s->t_count[ev.cls] += 1;
      s->t_ms[ev.cls] += ms;
    }
    s->event_pool.push_back(ev.a);
    s->event_pool.push_back(ev.b);
  }
  s->events.clear();
}

template <typename T>
ib_status run_body_ops(ib_solver* s) {
  HIPCHK(launch_body_ops<T>(s->fa, s->stream));
  return IB_OK;
}

ib_status map_flags(ib_solver* s, int code) {
  if (code == 1) {
    s->last_error = "a body point left the sub-domain";
    return IB_ERR_OUT_OF_SUBDOMAIN;
  }
  if (code == 2) {
    s->last_error = "delta support reaches the level-0 boundary";
    return IB_ERR_NEAR_BOUNDARY;
  }
  if (code == 3) {
    s->last_error = "singular or non-finite Schur matrix";
    return IB_ERR_NONFINITE;
  }
  if (code == FLAG_BARRIER) {
    s->last_error = "a device-wide barrier timed out";
    return IB_ERR_HIP;
  }
  return IB_OK;
}

// Device body data, the stationary Schur inverse or B' (Algorithm 1).
// Dense inverse X of the n x n matrix M (device, pitch pm) by Newton-Schulz iterations
// X <- X (2I - M X) on the FP64 matrix cores, from X0 = M^T / (|M|_1 |M|_inf) (which
// makes the iteration converge for any nonsingular M); mh is M on the host (for the
// norms and X0).  Stops when max |M X - I| < 1e-13, or fails (returns false) after 100
// iterations or on a non-finite or diverging residual.
bool newton_schulz_inverse(ib_solver* s, const double* M, double* X, int n, int pm,
                           const std::vector<double>& mh, ib_status* err) {
  *err = IB_OK;
  double n1 = 0.0, ninf = 0.0;
  std::vector<double> col(n, 0.0);
  for (int i = 0; i < n; ++i) {
    double r = 0.0;
    for (int j = 0; j < n; ++j) {
      const double v = std::fabs(mh[(size_t)i * pm + j]);
      r += v;
      col[j] += v;
    }
    ninf = std::max(ninf, r);
  }
  for (int j = 0; j < n; ++j) n1 = std::max(n1, col[j]);
  if (!(n1 > 0.0) || !(ninf > 0.0)) return false;
  const double alpha = 1.0 / (n1 * ninf);
  std::vector<double> x0((size_t)n * pm, 0.0);
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j) x0[(size_t)i * pm + j] = alpha * mh[(size_t)j * pm + i];
  double* W = static_cast<double*>(dalloc(s, (size_t)n * pm * 8));
  double* Y = static_cast<double*>(dalloc(s, (size_t)n * pm * 8));
  double* r = static_cast<double*>(dalloc(s, 8));
  if (!W || !Y || !r) {
    *err = IB_ERR_OOM;
    return false;
  }
  auto fail = [&](hipError_t e) {
    *err = hip_fail(s, e, "Newton-Schulz inverse");
    return false;
  };
  hipError_t e = hipMemcpy(X, x0.data(), x0.size() * 8, hipMemcpyHostToDevice);
  if (e != hipSuccess) return fail(e);
  double* cur = X;
  double* nxt = Y;
  double prev = 1e300, res = 1e300;
  bool ok = false;
  for (int it = 0; it < 100; ++it) {
    if ((e = launch_gemm64(M, cur, W, n, pm, 1, s->stream)) != hipSuccess) return fail(e);
    if ((e = hipMemsetAsync(r, 0, 8, s->stream)) != hipSuccess) return fail(e);
    if ((e = launch_eye_resid(W, pm, n, r, s->stream)) != hipSuccess) return fail(e);  // W - I = I - M X
    if ((e = hipMemcpyAsync(&res, r, 8, hipMemcpyDeviceToHost, s->stream)) != hipSuccess) return fail(e);
    if ((e = hipStreamSynchronize(s->stream)) != hipSuccess) return fail(e);
    if (!std::isfinite(res) || (it > 40 && res > prev)) break;
    if (res < 1e-13) {
      ok = true;
      break;
    }
    prev = res;
    if ((e = launch_gemm64(cur, W, nxt, n, pm, 0, s->stream)) != hipSuccess) return fail(e);
    std::swap(cur, nxt);
  }
  if (ok && cur != X) {
    e = hipMemcpyAsync(X, cur, (size_t)n * pm * 8, hipMemcpyDeviceToDevice, s->stream);
    if (e != hipSuccess) return fail(e);
    if ((e = hipStreamSynchronize(s->stream)) != hipSuccess) return fail(e);
  }
  dfree(s, W);
  dfree(s, Y);
  dfree(s, r);
  return ok;
}

// The offline operator for `key`: the imported one (which must match), a cached one, or
// a new one from `build`, which then enters the cache.
template <typename F>
ib_status acquire_op(ib_solver* s, const std::vector<double>& key, F build) {
  if (s->imported) {
    if (s->imported->key != key) {
      s->last_error = "imported operator does not match this problem";
      return IB_ERR_ARG;
    }
    s->op = s->imported;
    s->op_source = 2;
    return IB_OK;
  }
  OpPtr p = op_cache_get(key);
  if (p) {
    s->op = p;
    s->op_source = 1;
    return IB_OK;
  }
  auto d = std::make_shared<OpData>();
  d->key = key;
  ib_status st = build(*d);
  op_cache_done(key, st ? nullptr : d);
  if (st) return st;
  s->op = d;
  s->op_source = 0;
  return IB_OK;
}

// Poses of the rigid bodies in prescribed motion at time t (x, y, angle, vx, vy, omega from
// their callbacks, and the accelerations ax, ay, alpha_dd where given), and the frames of
// the torsional bodies mounted on them, into the device array the FSI kernels read; the
// staging alternates between two pinned sets, so a copy still pending from the previous
// step is not overwritten.
size_t pose_doubles(const ib_solver* s) { return (size_t)6 * s->nmov + (size_t)MOUNT_W * s->nmount; }

ib_status driver_pose(ib_solver* s, HostBody& hb, double t, double* q) {
  for (int e = 0; e < 9; ++e) q[e] = e < 6 ? 0.0 : std::nan("");
  hb.motion(t, q, hb.motion_ctx);
  for (int e = 0; e < 6; ++e)
    if (!std::isfinite(q[e])) {
      s->last_error = "non-finite pose from a motion callback";
      return IB_ERR_NONFINITE;
    }
  return IB_OK;
}

ib_status update_poses(ib_solver* s, double t) {
  if (!s->nmov) return IB_OK;
  const size_t w = pose_doubles(s);
  double* hp = s->hpose + w * (s->step & 1);
  int k = 0;
  for (auto& hb : s->bodies) {
    if (hb.kind != BODY_MOVING) continue;
    double q[9];
    ib_status st = driver_pose(s, hb, t, q);
    if (st) return st;
    for (int e = 0; e < 6; ++e) hp[6 * k + e] = q[e];
    for (int e = 0; e < 9; ++e) hb.pose[e] = q[e];
    ++k;
  }
  int j = 0;
  for (auto& hb : s->bodies) {
    if (hb.kind != BODY_TORSIONAL || hb.driver < 0) continue;
    const HostBody& d = s->bodies[hb.driver];
    for (int e = 6; e < 9; ++e)
      if (!std::isfinite(d.pose[e])) {
        s->last_error = "the driver of a mounted torsional body gives no accelerations";
        return IB_ERR_NONFINITE;
      }
    mount_frame(hb, d.pose, hp + 6 * s->nmov + (size_t)MOUNT_W * j);
    ++j;
  }
  HIPCHK(hipMemcpyAsync(const_cast<double*>(s->fa.poses), hp, w * 8, hipMemcpyHostToDevice,
                        s->stream));
  return IB_OK;
}

template <typename T>
ib_status prepare_bodies(ib_solver* s) {
  const int n = s->n;
  LevelState& L0 = s->lv[0];
  const double h = L0.h;
  const double x0 = s->cfg.cx - 0.5 * n * h, y0 = s->cfg.cy - 0.5 * n * h;
  // ---- host-side layout
  std::vector<BodyDev> bd;
  std::vector<double> rigid_xy, rigid_ub, tors, chi, dmass, l0v, beta0v, appxy;
  int pt = 0, app = 0, ntors = 0, dof = 0, nmov = 0;
  int64_t yoff = 0;
  bool any_moving = false;
  s->ds_rows.clear();
  int nmount = 0;
  for (auto& hb : s->bodies) {
    BodyDev b{};
    b.moff = -1;
    b.kind = hb.kind;
    b.npts = hb.m;
    b.pt0 = pt;
    b.ds = hb.ds;
    for (int k = 0; k < 2 * hb.m; ++k) s->ds_rows.push_back(hb.ds);
    // rigid geometry array is indexed by global point
    rigid_xy.resize(2 * (pt + hb.m), 0.0);
    rigid_ub.resize(2 * (pt + hb.m), 0.0);
    if (hb.kind == BODY_RIGID) {
      for (int k = 0; k < 2 * hb.m; ++k) rigid_xy[2 * pt + k] = hb.xy[k];
      if (!hb.ub.empty()) {
        b.has_ub = 1;
        for (int k = 0; k < 2 * hb.m; ++k) rigid_ub[2 * pt + k] = hb.ub[k];
      }
      b.app0 = app;
      for (int k = 0; k < 2 * hb.m; ++k) appxy.push_back(hb.xy[k]);
      app += hb.m;
    } else if (hb.kind == BODY_MOVING) {
      any_moving = true;
      b.tors = nmov++;
      for (int k = 0; k < 2 * hb.m; ++k) rigid_xy[2 * pt + k] = hb.xy[k];  // body frame
    } else if (hb.kind == BODY_TORSIONAL) {
      any_moving = true;
      b.tors = ntors++;
      b.hx = hb.hx;
      b.hy = hb.hy;
      b.theta0 = hb.theta0;
      b.inertia = hb.inertia;
      b.stiffness = hb.stiffness;
      b.damping = hb.damping;
      double g0 = 0.0;  // g at t = 0 (for the initial angular acceleration)
      if (hb.driver >= 0) {
        // mounted: frame offset fixed below, once the moving bodies are counted
        b.moff = nmount++;
        b.mass = hb.mass;
        b.cg = hb.cg;
        double q[9], fr[MOUNT_W];
        ib_status pst = driver_pose(s, s->bodies[hb.driver], 0.0, q);
        if (pst) return pst;
        if (!std::isfinite(q[6]) || !std::isfinite(q[7]) || !std::isfinite(q[8])) {
          s->last_error = "the driver of a mounted torsional body gives no accelerations";
          return IB_ERR_NONFINITE;
        }
        mount_frame(hb, q, fr);
        g0 = mount_g(hb, fr, hb.theta);
      }
      const double phidot = (g0 - hb.damping * hb.phi - hb.stiffness * hb.theta) / hb.inertia;
      const double st[TS_COUNT] = {hb.theta, hb.phi, phidot, hb.theta, 0.0};
      tors.insert(tors.end(), st, st + TS_COUNT);
    } else {
      any_moving = true;
      b.dof0 = dof;
      b.yoff = yoff;
      yoff += (int64_t)3 * hb.m * (2 * hb.m + 1);
      b.mass = hb.mass;
      b.ei = hb.ei;
      b.ea = hb.ea;
      const int m = hb.m;
      chi.resize(dof + 3 * m, 0.0);
      dmass.resize(dof + 3 * m, 0.0);
      l0v.resize(dof / 3 + m, 0.0);
      beta0v.resize(dof / 3 + m, 0.0);
      for (int k = 0; k < m; ++k) {
        chi[dof + 3 * k] = hb.xy0[2 * k];
        chi[dof + 3 * k + 1] = hb.xy0[2 * k + 1];
        chi[dof + 3 * k + 2] = hb.rot0[k];
      }
      for (int e = 0; e < m - 1; ++e) {
        const double dx = hb.xy_ref[2 * e + 2] - hb.xy_ref[2 * e];
        const double dy = hb.xy_ref[2 * e + 3] - hb.xy_ref[2 * e + 1];
        const double le = std::sqrt(dx * dx + dy * dy);
        l0v[dof / 3 + e] = le;
        beta0v[dof / 3 + e] = std::atan2(dy, dx);
        const double me = hb.mass * le;
        for (int node = e; node <= e + 1; ++node) {
          dmass[dof + 3 * node] += 0.5 * me;
          dmass[dof + 3 * node + 1] += 0.5 * me;
          dmass[dof + 3 * node + 2] += me * le * le / 105.0;
        }
      }
      dof += 3 * m;
    }
    bd.push_back(b);
    pt += hb.m;
  }
  for (auto& b : bd)
    if (b.moff >= 0) b.moff = 6 * nmov + MOUNT_W * b.moff;  // frames follow the poses
  s->npts = pt;
  s->nf = 2 * pt;
  s->ntors = ntors;
  s->ndof = dof;
  // ---- mode
  int mode = s->cfg.schur_mode;
  if (mode == IB_SCHUR_AUTO) mode = s->has_sd ? IB_SCHUR_SUBDOMAIN : IB_SCHUR_EXACT;
  s->use_sd = mode == IB_SCHUR_SUBDOMAIN;
  if (s->use_sd && !s->has_sd) {
    s->last_error = "sub-domain mode needs ib_set_subdomain";
    return IB_ERR_STATE;
  }
  if (s->use_sd && s->cfg.delta != IB_DELTA_ROMA3) {
    s->last_error = "the 4-point delta kernel is available with the exact operator only";
    return IB_ERR_ARG;
  }
  s->stationary = !s->use_sd && !any_moving;
  s->exact_moving = !s->use_sd && any_moving;
  if (!s->stationary && s->nf > 0) {
    // the refinement's device-wide barrier needs all its workgroups resident at once
    int have = 0, need = 0;
    s->lu_always = !refine_coresident(s->nf, &have, &need);
  }
  for (auto& hb : s->bodies)
    if (hb.kind == BODY_DEFORMABLE && 3 * hb.m - 3 > 600) {
      s->last_error = "deformable body with more than 201 nodes";
      return IB_ERR_ARG;
    }
  // ---- sub-domain geometry: each rectangle snapped outwards to vertices, their vertex
  // grids one after another; each moving body interpolates on one rectangle
  if (s->use_sd) {
    const double tol = 1e-9;
    ib::SdBoxes& q = s->sdb;
    q = ib::SdBoxes{};
    q.n = (int)s->sd_rects.size();
    int tot = 0;
    s->sd_ilo = s->sd_jlo = n;
    s->sd_ihi = s->sd_jhi = 0;
    std::vector<std::array<int, 4>> ext(q.n);
    for (int k = 0; k < q.n; ++k) {
      const auto& r = s->sd_rects[k];
      const int i0 = (int)std::floor((r[0] - x0) / h + tol), i1 = (int)std::ceil((r[1] - x0) / h - tol);
      const int j0 = (int)std::floor((r[2] - y0) / h + tol), j1 = (int)std::ceil((r[3] - y0) / h - tol);
      if (i0 < 2 || j0 < 2 || i1 > n - 2 || j1 > n - 2) {
        s->last_error = "sub-domain reaches the level-0 boundary";
        return IB_ERR_NEAR_BOUNDARY;
      }
      q.i0[k] = i0;
      q.j0[k] = j0;
      q.npx[k] = i1 - i0 + 1;
      q.npy[k] = j1 - j0 + 1;
      q.off[k] = tot;
      tot += q.npx[k] * q.npy[k];
      ext[k] = {i0, i1, j0, j1};
      s->sd_ilo = std::min(s->sd_ilo, i0);
      s->sd_ihi = std::max(s->sd_ihi, i1);
      s->sd_jlo = std::min(s->sd_jlo, j0);
      s->sd_jhi = std::max(s->sd_jhi, j1);
    }
    s->sd_ngrid = tot;
    s->sd_total = s->sd_ngrid + app;
    // a torsional or deformable body uses the first rectangle that holds all its points at
    // the start; bodies in prescribed motion and plates mounted on them use the first
    auto holds = [&](int k, double px, double py) {
      const double rx = (px - (x0 + q.i0[k] * h)) / h, ry = (py - (y0 + q.j0[k] * h)) / h;
      return rx >= -tol && ry >= -tol && rx <= q.npx[k] - 1 + tol && ry <= q.npy[k] - 1 + tol;
    };
    for (size_t bi = 0; bi < s->bodies.size(); ++bi) {
      const HostBody& hb = s->bodies[bi];
      int box = 0;
      std::vector<double> pts;
      if (hb.kind == BODY_TORSIONAL && hb.driver < 0) {
        for (int j = 0; j < hb.m; ++j) {
          pts.push_back(hb.hx + j * hb.ds * std::cos(hb.theta0 + hb.theta));
          pts.push_back(hb.hy + j * hb.ds * std::sin(hb.theta0 + hb.theta));
        }
      } else if (hb.kind == BODY_DEFORMABLE) {
        pts = hb.xy0;
      }
      if (!pts.empty()) {
        box = -1;
        for (int k = 0; k < q.n && box < 0; ++k) {
          bool all = true;
          for (size_t e = 0; e + 1 < pts.size() && all; e += 2) all = holds(k, pts[e], pts[e + 1]);
          if (all) box = k;
        }
        if (box < 0) {
          s->last_error = "a body lies outside every sub-domain rectangle";
          return IB_ERR_OUT_OF_SUBDOMAIN;
        }
      }
      bd[bi].sdbox = box;
    }
  }
  // rows and columns the body operators and the spread can touch
  {
    double xmin = 1e300, xmax = -1e300, ymin = 1e300, ymax = -1e300;
    auto acc = [&](double x, double y) {
      xmin = std::min(xmin, x); xmax = std::max(xmax, x);
      ymin = std::min(ymin, y); ymax = std::max(ymax, y);
    };
    for (auto& hb : s->bodies) if (hb.kind == BODY_RIGID) for (int k = 0; k < hb.m; ++k) acc(hb.xy[2 * k], hb.xy[2 * k + 1]);
    if (s->use_sd) {
      acc(x0 + s->sd_ilo * h, y0 + s->sd_jlo * h);
      acc(x0 + s->sd_ihi * h, y0 + s->sd_jhi * h);
    }
    if (xmin > xmax) { xmin = xmax = s->cfg.cx; ymin = ymax = s->cfg.cy; }
    s->bilo = std::max(1, (int)std::floor((xmin - x0) / h) - 4);
    s->bihi = std::min(n - 1, (int)std::ceil((xmax - x0) / h) + 4);
    s->blo = std::max(1, (int)std::floor((ymin - y0) / h) - 4);
    s->bhi = std::min(n - 1, (int)std::ceil((ymax - y0) / h) + 4);
    if (s->exact_moving) {
      // moving bodies without a sub-domain may go anywhere on level 0
      s->bilo = s->blo = 1;
      s->bihi = s->bhi = n - 1;
    }
  }
  // ---- device arrays
  auto up = [&](const std::vector<double>& v) -> double* {
    double* p = static_cast<double*>(dalloc(s, std::max<size_t>(1, v.size()) * 8));
    if (p && !v.empty()) (void)hipMemcpy(p, v.data(), v.size() * 8, hipMemcpyHostToDevice);
    return p;
  };
  FsiArgs& a = s->fa;
  a = FsiArgs{};
  BodyDev* dbodies = static_cast<BodyDev*>(dalloc(s, bd.size() * sizeof(BodyDev)));
  HIPCHK(hipMemcpy(dbodies, bd.data(), bd.size() * sizeof(BodyDev), hipMemcpyHostToDevice));
  a.bodies = dbodies;
  a.nbodies = (int)bd.size();
  a.npts = s->npts;
  a.nf = s->nf;
  a.ntors = ntors;
  a.n = n;
  a.ps = s->pitch;
  a.h = h;
  a.x0 = x0;
  a.y0 = y0;
  a.ux = s->cfg.u_inf[0] * h;
  a.uy = s->cfg.u_inf[1] * h;
  a.dt = s->cfg.dt;
  a.delta_kind = s->cfg.delta;
  a.sstar = s->sstar;
  a.fp64 = s->fp64;
  a.use_sd = s->use_sd;
  a.sdb = s->sdb;
  a.sd_ngrid = s->sd_ngrid;
  a.sd_total = s->sd_total;
  a.app_xy = up(appxy);
  a.rigid_xy = up(rigid_xy);
  a.rigid_ub = up(rigid_ub);
  s->nmov = nmov;
  s->nmount = nmount;
  a.poses = nullptr;
  if (nmov) {
    a.poses = static_cast<double*>(dalloc(s, pose_doubles(s) * 8));
    if (!a.poses) return IB_ERR_OOM;
    if (!s->hpose) HIPCHK(hipHostMalloc(reinterpret_cast<void**>(&s->hpose), 2 * pose_doubles(s) * 8,
                                        hipHostMallocDefault));
    ib_status pst = update_poses(s, (s->step + 1) * s->cfg.dt);
    if (pst) return pst;
    HIPCHK(hipStreamSynchronize(s->stream));
  }
  const int nf = s->nf;
  a.st_base = static_cast<int*>(dalloc(s, (size_t)nf * 3 * 4));
  a.st_w = static_cast<double*>(dalloc(s, (size_t)nf * 16 * 8));
  a.p_idx = static_cast<int*>(dalloc(s, (size_t)nf * 4 * 4));
  a.p_w = static_cast<double*>(dalloc(s, (size_t)nf * 4 * 8));
  a.act = nullptr;
  if (s->use_sd) {
    if ((size_t)nf * SCHUR_LDS_PER_ROW > SCHUR_LDS_MAX) {
      s->last_error = "too many body points for the sub-domain Schur assembly";
      return IB_ERR_CAPACITY;
    }
    a.act = static_cast<int*>(dalloc(s, (size_t)2 * s->sd_total * 4));
    if (!a.act) return IB_ERR_OOM;
    HIPCHK(hipMemset(a.act, 0xff, (size_t)2 * s->sd_total * 4));
  }
  a.pos = static_cast<double*>(dalloc(s, (size_t)s->npts * 2 * 8));
  a.ustar = static_cast<double*>(dalloc(s, (size_t)nf * 8));
  s->f = static_cast<double*>(dalloc(s, (size_t)nf * 8));
  s->rhs = static_cast<double*>(dalloc(s, (size_t)nf * 8));
  a.f = s->f;
  a.rhs = s->rhs;
  a.pm = round_up(nf, 8);
  a.M = static_cast<double*>(dalloc(s, (size_t)nf * a.pm * 8 + 8));
  if (!s->stationary) {
    const size_t mb = (size_t)nf * a.pm * 8 + 8;
    s->Minv = static_cast<double*>(dalloc(s, mb));
    s->Xn = static_cast<double*>(dalloc(s, mb));
    s->W = static_cast<double*>(dalloc(s, mb));
    s->Mtmp = static_cast<double*>(dalloc(s, mb));
    s->rinfo = static_cast<double*>(dalloc(s, refine_ws_doubles(nf, REFINE_MAXIT) * 8));
    if (!s->Minv || !s->Xn || !s->W || !s->Mtmp || !s->rinfo) return IB_ERR_OOM;
    // the refinement's barrier counters and norms start at zero (each launch leaves them so)
    HIPCHK(hipMemset(s->rinfo, 0, refine_ws_doubles(nf, REFINE_MAXIT) * 8));
    s->x_valid = false;
  }
  a.tors = up(tors);
  a.chi = up(chi);
  a.zeta = up(std::vector<double>(chi.size(), 0.0));
  a.zetadot = up(std::vector<double>(chi.size(), 0.0));
  a.chi_new = up(chi);
  a.dmass = up(dmass);
  a.l0 = up(l0v);
  a.beta0 = up(beta0v);
  size_t yw = 0;
  for (auto& hb : s->bodies) if (hb.kind == BODY_DEFORMABLE) yw += (size_t)3 * hb.m * (2 * hb.m + 1);
  a.ywork = static_cast<double*>(dalloc(s, std::max<size_t>(1, yw) * 8));
  s->ctl = dalloc(s, 64);
  if (!a.st_base || !a.st_w || !a.M || !s->f || !s->ctl) return IB_ERR_OOM;
  s->flags = static_cast<int*>(s->ctl);
  s->gate = s->flags + FsiCtl::GATE;
  s->delta = reinterpret_cast<double*>(static_cast<char*>(s->ctl) + 8);
  s->rout = reinterpret_cast<double*>(static_cast<char*>(s->ctl) + 16);
  a.flags = s->flags;
  a.delta = s->delta;
  HIPCHK(hipMemset(s->ctl, 0, 64));
  if (!s->hctl) {
    HIPCHK(hipHostMalloc(&s->hctl, 64, hipHostMallocDefault));
    std::memset(s->hctl, 0, 64);
    s->hflags = static_cast<int*>(s->hctl);
    s->hdelta = reinterpret_cast<double*>(static_cast<char*>(s->hctl) + 8);
    s->hrinfo = reinterpret_cast<double*>(static_cast<char*>(s->hctl) + 16);
  }
  if (dof > 0) HIPCHK(launch_beam_init(a, s->stream));
  // operator at the initial configuration
  a.iter = 0;
  ib_status st = run_body_ops<T>(s);
  if (st) return st;
  HIPCHK(hipStreamSynchronize(s->stream));
  HIPCHK(hipMemcpy(s->hflags, s->flags, 8, hipMemcpyDeviceToHost));
  if ((st = map_flags(s, s->hflags[0]))) return st;
  // ---- offline operator
  OffRows geo{};
  geo.n = n;
  geo.h = h;
  geo.x0 = x0;
  geo.y0 = y0;
  if (s->exact_moving) {
    // buffers for rebuilding the exact flow block at every FSI iterate
    s->xrows = geo;
    s->xrows.kind = 0;
    s->xrows.st_base = a.st_base;
    s->xrows.st_w = a.st_w;
    const int slots = std::min(offline_slots(s, nf), nf);
    if ((st = offline_alloc(s, s->xo, slots, nf))) return st;
    s->gx = static_cast<double*>(dalloc(s, (size_t)nf * a.pm * 8));
    if (!s->gx) return IB_ERR_OOM;
    a.gx = s->gx;
  }
  if (s->stationary) {
    OffRows rows = geo;
    rows.kind = 0;
    rows.st_base = a.st_base;
    rows.st_w = a.st_w;
    // the cached product is M^{-1} itself (stationary bodies: the whole Schur inverse
    // depends only on the key, which includes the points' arc lengths)
    double* G = a.M;  // G then M in place
    const int tlo = std::max(1, s->blo), thi = std::min(n - 1, s->bhi);
    std::vector<double> key = {0.0, (double)n, h, x0, y0, s->cfg.dt, s->cfg.re, (double)nf,
                               (double)a.pm};
    key.insert(key.end(), rigid_xy.begin(), rigid_xy.end());
    key.insert(key.end(), s->ds_rows.begin(), s->ds_rows.end());
    key.push_back((double)s->cfg.delta);  // the delta kernel shapes E
    s->Minv = static_cast<double*>(dalloc(s, (size_t)nf * a.pm * 8 + 8));
    if (!s->Minv) return IB_ERR_OOM;
    st = acquire_op(s, key, [&](OpData& d) -> ib_status {
      Offline w;
      const int slots = std::min(offline_slots(s, nf), nf);
      ib_status e = offline_alloc(s, w, slots, nf);
      if (e) return e;
      std::vector<double> hv((size_t)slots * nf);
      std::vector<double> gm((size_t)nf * a.pm, 0.0);
      for (int c0 = 0; c0 < nf; c0 += slots) {
        if ((e = offline_columns(s, w, rows, c0, nf, rows, nf, tlo, thi))) return e;
        const int ns = std::min(slots, nf - c0);
        HIPCHK(hipMemcpyAsync(hv.data(), w.vals, (size_t)ns * nf * 8, hipMemcpyDeviceToHost,
                              s->stream));
        HIPCHK(hipStreamSynchronize(s->stream));
        for (int b = 0; b < ns; ++b)
          for (int t = 0; t < nf; ++t) gm[(size_t)t * a.pm + c0 + b] = hv[(size_t)b * nf + t];
      }
      offline_free(s, w);
      // M = (dt / h^2) G diag(ds), on the host too (for the inverse's starting point)
      const double sc = s->cfg.dt / (h * h);
      for (int i = 0; i < nf; ++i)
        for (int j = 0; j < nf; ++j) gm[(size_t)i * a.pm + j] *= sc * s->ds_rows[j];
      HIPCHK(hipMemcpy(G, gm.data(), gm.size() * 8, hipMemcpyHostToDevice));
      // inverse: Newton-Schulz on the matrix cores; LU with partial pivoting if that fails
      if (!newton_schulz_inverse(s, G, s->Minv, nf, a.pm, gm, &e)) {
        if (e) return e;
        std::vector<double> eye((size_t)nf * a.pm, 0.0);
        for (int k = 0; k < nf; ++k) eye[(size_t)k * a.pm + k] = 1.0;
        HIPCHK(hipMemcpy(s->Minv, eye.data(), eye.size() * 8, hipMemcpyHostToDevice));
        HIPCHK(launch_lu_solve(G, a.pm, s->Minv, a.pm, nf, nf, s->flags, s->stream));
        HIPCHK(hipStreamSynchronize(s->stream));
        HIPCHK(hipMemcpy(s->hflags, s->flags, 8, hipMemcpyDeviceToHost));
        if ((e = map_flags(s, s->hflags[0]))) return e;
      }
      d.val.resize((size_t)nf * a.pm);
      HIPCHK(hipMemcpy(d.val.data(), s->Minv, d.val.size() * 8, hipMemcpyDeviceToHost));
      return IB_OK;
    });
    if (st) return st;
    if (s->op_source != 0) {
      if (s->op->val.size() != (size_t)nf * a.pm) {
        s->last_error = "offline operator has the wrong size";
        return IB_ERR_ARG;
      }
      HIPCHK(hipMemcpy(s->Minv, s->op->val.data(), s->op->val.size() * 8, hipMemcpyHostToDevice));
    }
    a.Minv = s->Minv;
  } else if (s->use_sd) {
    OffRows rows = geo;
    rows.kind = 1;
    rows.sdb = s->sdb;
    rows.sd_ngrid = s->sd_ngrid;
    rows.sd_total = s->sd_total;
    rows.app_xy = a.app_xy;
    const int nsd = 2 * s->sd_total;
    // target rows: the sub-domain vertices' windows and the appended points' windows
    int tlo = s->sd_jlo - 2, thi = s->sd_jhi + 3;
    for (size_t k = 0; k < appxy.size() / 2; ++k) {
      const int jj = (int)std::floor((appxy[2 * k + 1] - y0) / h);
      tlo = std::min(tlo, jj - 3);
      thi = std::max(thi, jj + 4);
    }
    tlo = std::max(1, tlo);
    thi = std::min(n - 1, thi);
    std::vector<double> key = {1.0, (double)n, h, x0, y0, s->cfg.dt, s->cfg.re, s->cfg.drop_tol,
                               (double)s->sdb.n};
    for (int k = 0; k < s->sdb.n; ++k)
      for (double v : {(double)s->sdb.i0[k], (double)s->sdb.j0[k], (double)s->sdb.npx[k],
                       (double)s->sdb.npy[k]})
        key.push_back(v);
    key.push_back((double)appxy.size());
    key.insert(key.end(), appxy.begin(), appxy.end());
    st = acquire_op(s, key, [&](OpData& d) -> ib_status {
      Offline w;
      const int slots = std::min(offline_slots(s, nsd), nsd);
      ib_status e = offline_alloc(s, w, slots, nsd);
      if (e) return e;
      int* ccol = static_cast<int*>(dalloc(s, (size_t)slots * nsd * 4));
      double* cval = static_cast<double*>(dalloc(s, (size_t)slots * nsd * 8));
      int* counts = static_cast<int*>(dalloc(s, (size_t)slots * 4));
      int* gcol = static_cast<int*>(dalloc(s, (size_t)slots * nsd * 4));
      double* gval = static_cast<double*>(dalloc(s, (size_t)slots * nsd * 8));
      if (!ccol || !cval || !counts || !gcol || !gval) return IB_ERR_OOM;
      d.ptr.assign(1, 0);
      std::vector<int> hcounts(slots);
      for (int c0 = 0; c0 < nsd; c0 += slots) {
        if ((e = offline_columns(s, w, rows, c0, nsd, rows, nsd, tlo, thi))) return e;
        const int ns = std::min(slots, nsd - c0);
        HIPCHK(launch_filter_compact(w.vals, nsd, c0, nsd, ns, s->cfg.drop_tol, ccol, cval, counts,
                                     s->stream));
        HIPCHK(launch_gather_batch(ccol, cval, nsd, counts, ns, gcol, gval, s->stream));
        HIPCHK(hipMemcpyAsync(hcounts.data(), counts, (size_t)ns * 4, hipMemcpyDeviceToHost,
                              s->stream));
        HIPCHK(hipStreamSynchronize(s->stream));
        int64_t tot = 0;
        for (int b = 0; b < ns; ++b) tot += hcounts[b];
        const size_t old = d.col.size();
        d.col.resize(old + tot);
        d.val.resize(old + tot);
        HIPCHK(hipMemcpy(d.col.data() + old, gcol, (size_t)tot * 4, hipMemcpyDeviceToHost));
        HIPCHK(hipMemcpy(d.val.data() + old, gval, (size_t)tot * 8, hipMemcpyDeviceToHost));
        for (int b = 0; b < ns; ++b) d.ptr.push_back(d.ptr.back() + hcounts[b]);
      }
      dfree(s, ccol);
      dfree(s, cval);
      dfree(s, counts);
      dfree(s, gcol);
      dfree(s, gval);
      offline_free(s, w);
      return IB_OK;
    });
    if (st) return st;
    const OpData& op = *s->op;
    if ((int64_t)op.ptr.size() != (int64_t)nsd + 1) {
      s->last_error = "offline operator has the wrong number of rows";
      return IB_ERR_ARG;
    }
    s->bp_nnz = (int64_t)op.col.size();
    int64_t* dptr = static_cast<int64_t*>(dalloc(s, op.ptr.size() * 8));
    int32_t* dcol = static_cast<int32_t*>(dalloc(s, std::max<size_t>(1, op.col.size()) * 4));
    double* dval = static_cast<double*>(dalloc(s, std::max<size_t>(1, op.val.size()) * 8));
    if (!dptr || !dcol || !dval) return IB_ERR_OOM;
    HIPCHK(hipMemcpy(dptr, op.ptr.data(), op.ptr.size() * 8, hipMemcpyHostToDevice));
    if (!op.col.empty()) {
      HIPCHK(hipMemcpy(dcol, op.col.data(), op.col.size() * 4, hipMemcpyHostToDevice));
      HIPCHK(hipMemcpy(dval, op.val.data(), op.val.size() * 8, hipMemcpyHostToDevice));
    }
    a.bp_ptr = dptr;
    a.bp_col = dcol;
    a.bp_val = dval;
  }
  return IB_OK;
}

template <typename T>
ib_status do_prepare(ib_solver* s) {
  auto t0 = std::chrono::steady_clock::now();
  ib_status st = init_streamfunction<T>(s);
  if (st) return st;
  if (!s->bodies.empty()) {
    st = prepare_bodies<T>(s);
    if (st) return st;
  }
  HIPCHK(hipStreamSynchronize(s->stream));
  s->prepare_seconds =
      std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  return IB_OK;
}

// --------------------------------------------------------------------- step

// One FSI iteration (the loop body of Algorithm 2): body operators and u*, the structure's
// right-hand side, the beam Jacobian solves, the Schur matrix (eqs. (17), (37)), the inverse
// it is solved with (fresh LU, or one Newton-Schulz refresh at the first iteration of a
// step), the refined stress solve and the structure update.  With a.gate set every kernel
// skips itself once the step's iterations have converged or stopped on the device.
// Whether FSI iteration `it` refreshes the approximate inverse before its stress solve.
bool refresh_at(const ib_solver* s, int it) {
  if (s->refresh_mode == 1) return true;
  if (s->refresh_mode == 0) return it == 0;
  if (s->nf <= REFRESH_ALL_NF) return true;
  return it == 0 && s->hrinfo != nullptr && s->hrinfo[1] > REFRESH_SWEEPS;
}

// Whether the refinement of FSI iteration `it` starts from the stresses in s->f: the previous
// iterate's, or at a step's first iteration the previous step's (every completed step leaves
// a converged solve there); not after a refinement that stopped contracting.
bool refine_guess(const ib_solver* s, int it) {
  return (it > 0 || s->step > 0) && !s->x_valid_retry;
}

template <typename T>
ib_status fsi_iteration(ib_solver* s, const FsiArgs& a0, int it, int K = 0) {
  FsiArgs a = a0;
  a.iter = it;
  const int n = s->n, nf = s->nf;
  TimeScope ts(s, IB_K_FSI);
  // the body operators and the first deformable body's beam solves share one launch
  int fused = -1;
  for (size_t bi = 0; bi < s->bodies.size(); ++bi)
    if (s->bodies[bi].kind == BODY_DEFORMABLE) {
      if (fused < 0) {
        fused = (int)bi;
        HIPCHK(launch_ops_beam<T>(a, fused, s->bodies[bi].m, s->stream));
      } else {
        HIPCHK(launch_beam(a, (int)bi, s->bodies[bi].m, s->stream));
      }
    }
  if (fused < 0) HIPCHK(launch_body_ops<T>(a, s->stream));
  if (s->exact_moving) {
    // the exact flow block at this iterate: one point-source solve per body row
    for (int c0 = 0; c0 < nf; c0 += s->xo.nslots) {
      ib_status e = offline_columns(s, s->xo, s->xrows, c0, nf, s->xrows, nf, 1, n - 1);
      if (e) return e;
      HIPCHK(launch_cols_to_matrix(s->xo.vals, nf, std::min(s->xo.nslots, nf - c0), c0, s->gx,
                                   a.pm, s->stream));
    }
  }
  HIPCHK(launch_schur_sd(a, s->stream));
  const size_t mb = (size_t)nf * a.pm * 8;
  if (s->lu_always || s->lu_step) {
    // the stress solve without a device-wide barrier: LU with partial pivoting of a copy
    HIPCHK(hipMemcpyAsync(s->Mtmp, a.M, mb, hipMemcpyDeviceToDevice, s->stream));
    HIPCHK(hipMemcpyAsync(s->f, s->rhs, (size_t)nf * 8, hipMemcpyDeviceToDevice, s->stream));
    HIPCHK(launch_lu_solve(s->Mtmp, a.pm, s->f, 1, nf, 1, s->flags, s->stream));
    HIPCHK(launch_update(a, it, K, s->cfg.newton_tol, s->cfg.newton_fixed_iter, s->stream));
    return IB_OK;
  }
  const bool fresh = !s->x_valid;
  if (fresh) {
    // fresh inverse of the current Schur matrix by LU on a copy
    HIPCHK(hipMemcpyAsync(s->Mtmp, a.M, mb, hipMemcpyDeviceToDevice, s->stream));
    HIPCHK(hipMemsetAsync(s->Minv, 0, mb, s->stream));
    HIPCHK(launch_identity(s->Minv, a.pm, nf, s->stream));
    HIPCHK(launch_lu_solve(s->Mtmp, a.pm, s->Minv, a.pm, nf, nf, s->flags, s->stream));
    s->x_valid = true;
    s->inverse_rebuilds++;
  }
  const double* X = s->Minv;
  double* xcopy = nullptr;
  if (!fresh && refresh_at(s, it)) {
    // one Newton-Schulz step towards the new matrix, X <- X (2I - M X), into Xn; the
    // refinement solves with it and copies it back to Minv as it loads it
    HIPCHK(launch_gemm64(a.M, s->Minv, s->W, nf, a.pm, 1, s->stream, a.gate));
    HIPCHK(launch_gemm64(s->Minv, s->W, s->Xn, nf, a.pm, 0, s->stream, a.gate));
    X = s->Xn;
    xcopy = s->Minv;
  }
  // the refinement and then, in the same launch, the structure update with the new stresses
  HIPCHK(launch_refine(a.M, a.pm, X, s->rhs, s->f, nf, REFINE_MAXIT, refine_guess(s, it),
                       s->rinfo, s->rout, s->flags, a.gate, xcopy, s->barrier_arg(), s->stream,
                       &a, it, K, s->cfg.newton_tol, s->cfg.newton_fixed_iter));
  return IB_OK;
}

// Corrector s_{n+1} = s* - dt K C^T E^T (ds/h) f on level 0 (eqs. (20), (40)); with `gate`
// set it runs only if the step's iterations converged on the device.  finish: the spread's
// launch also runs the structure finish (k_finish's work) in a workgroup of its own.
template <typename T>
ib_status corrector(ib_solver* s, const int* gate, bool finish = false) {
  const int n = s->n, P = s->pitch;
  LevelState& L0 = s->lv[0];
  FsiArgs a = s->fa;
  a.gate = gate;
  {
    TimeScope ts(s, IB_K_CORRECT);
    HIPCHK(launch_spread<T>(a, s->blo, s->bhi, s->bilo, s->bihi, static_cast<T*>(s->work2), P,
                            s->stream, finish));
    RowArgs<T> r{};
    r.in = static_cast<T*>(s->work2);
    r.out = static_cast<T*>(s->work2);
    r.pi = r.po = P;
    r.r0 = s->blo;
    r.r1 = s->bhi;
    r.gate = gate;
    HIPCHK(launch_rowdst<T>(r, n, 1, s->tw, s->stream));
  }
  ColArgs<T> c{};
  c.in = static_cast<T*>(s->work2);
  c.out = static_cast<T*>(s->work);
  c.pi = c.po = P;
  c.r0 = s->blo;
  c.r1 = s->bhi;
  c.alpha = (T)L0.alpha;
  c.scale = (T)(-s->cfg.dt * 4.0 / ((double)n * n));
  c.out2 = static_cast<T*>(s->workg);
  c.accumulate = 1;
  c.w0 = 1;
  c.w1 = n - 1;
  c.var = s->tune.col;
  c.gate = gate;
  TimeScope ts(s, IB_K_COL_SOLVE, true);
  c.ev0 = ts.b;
  c.ev1 = ts.e;
  HIPCHK(launch_col_solve<T>(c, n, 1, s->tw, s->lam, s->stream));
  return IB_OK;
}

// Whether this step's FSI iterations can be launched ahead of their convergence tests
// (device-side control, one host synchronisation per step).  The first use of the Schur
// inverse (LU) and the exact operator (host-driven column solves) stay on the host path.
bool fsi_ahead(const ib_solver* s) {
  return !s->stationary && !s->exact_moving && s->x_valid && s->fsi_ahead && !s->lu_always;
}

int fsi_ahead_count(const ib_solver* s) {
  const int fixed = s->cfg.newton_fixed_iter;
  const int kmax = s->cfg.newton_max_iter > 0 ? s->cfg.newton_max_iter : 20;
  if (fixed > 0) return std::min(fixed, kmax);
  return std::max(1, std::min(kmax, s->iters_last > 0 ? s->iters_last : 2));
}

// Launch the step's FSI iterations ahead: K iterations, each followed by the device-side
// convergence test, then the structure's finish and the corrector, all gated.
template <typename T>
ib_status fsi_launch_ahead(ib_solver* s, int K) {
  FsiArgs g = s->fa;
  g.gate = s->gate;
  for (int it = 0; it < K; ++it) {
    ib_status e = fsi_iteration<T>(s, g, it, K);  // k_update runs the convergence test
    if (e) return e;
  }
  return corrector<T>(s, s->gate, true);  // with the structure finish
}

// A refinement's device-wide barrier timed out (its workgroups were not all resident, e.g.
// next to other solvers' kernels): the step's FSI iterations are redone from the old
// structure state (the finish and corrector never ran) with LU solves, and the approximate
// inverse, which that refinement may have left half refreshed, is rebuilt at its next use.
ib_status begin_solve_fallback(ib_solver* s) {
  HIPCHK(launch_step_reset(s->flags, s->stream));
  s->lu_step = true;
  s->x_valid = false;
  s->x_valid_retry = false;
  s->solve_fallbacks++;
  return IB_OK;
}

// After the iterations launched ahead (and a synchronisation that brought the control block
// to the host): converged, or go on on the host from where the device stopped.  *resume
// receives the iteration to continue with, or -1 when the step's FSI part is complete.
ib_status fsi_after_ahead(ib_solver* s, int* resume) {
  *resume = -1;
  const int* hc = static_cast<const int*>(s->hctl);
  const int next = hc[FsiCtl::NEXT];
  if (hc[FsiCtl::GATE] == 1 && hc[FsiCtl::GATE + 1] == 0) {
    s->iters_last = next;
    s->delta_last = s->hdelta[0];
    s->iters_max = std::max(s->iters_max, s->iters_last);
    return IB_OK;
  }
  if (s->hflags[0] == FLAG_BARRIER) {
    ib_status e = begin_solve_fallback(s);
    if (e) return e;
    *resume = 0;
    return IB_OK;
  }
  ib_status st = map_flags(s, s->hflags[0]);
  if (st) return st;
  if (s->hflags[1]) {
    // the approximate inverse no longer contracts: rebuild it and redo that iteration
    s->x_valid = false;
    s->x_valid_retry = true;
  } else if (!std::isfinite(s->hdelta[0])) {
    s->last_error = "non-finite structure update";
    return IB_ERR_NONFINITE;
  }
  // clear the flags and gates (the host continues without them)
  HIPCHK(launch_step_reset(s->flags, s->stream));
  *resume = next;
  return IB_OK;
}

// FSI iterations with the convergence test on the host, from iteration `it0`, then the
// finish and the corrector.
template <typename T>
ib_status fsi_host(ib_solver* s, int it0) {
  FsiArgs& a = s->fa;
  const int fixed = s->cfg.newton_fixed_iter;
  const int kmax = s->cfg.newton_max_iter > 0 ? s->cfg.newton_max_iter : 20;
  int it = it0;
  for (;;) {
    if (s->stationary) {
      FsiArgs b = a;
      b.iter = 0;
      TimeScope ts(s, IB_K_FSI);
      HIPCHK(launch_body_ops<T>(b, s->stream));
      HIPCHK(launch_matvec(s->Minv, b.pm, s->rhs, s->f, s->nf, s->stream));
      s->iters_last = 1;
      s->delta_last = 0.0;
      break;
    }
    ib_status e = fsi_iteration<T>(s, a, it);
    if (e) return e;
    HIPCHK(hipMemcpyAsync(s->hctl, s->ctl, FsiCtl::BYTES, hipMemcpyDeviceToHost, s->stream));
    HIPCHK(hipStreamSynchronize(s->stream));
    if (s->hflags[0] == FLAG_BARRIER && !s->lu_step) {
      e = begin_solve_fallback(s);
      if (e) return e;
      it = 0;
      continue;
    }
    ib_status st = map_flags(s, s->hflags[0]);
    if (st) return st;
    if (s->hflags[1]) {
      // the approximate inverse no longer contracts: rebuild it and redo this iteration
      if (!s->x_valid_retry) {
        s->x_valid = false;
        s->x_valid_retry = true;
        HIPCHK(launch_step_reset(s->flags, s->stream));
        continue;
      }
      s->last_error = "Schur refinement did not converge";
      return IB_ERR_NONFINITE;
    }
    s->x_valid_retry = false;
    if (!std::isfinite(s->hdelta[0])) {
      s->last_error = "non-finite structure update";
      return IB_ERR_NONFINITE;
    }
    const bool done = fixed > 0 ? it + 1 >= fixed : s->hdelta[0] <= s->cfg.newton_tol;
    if (!done && it + 1 >= kmax) {
      s->iters_last = it + 1;
      s->delta_last = s->hdelta[0];
      s->last_error = "FSI iteration did not converge";
      return IB_ERR_NOT_CONVERGED;
    }
    if (done) {
      s->iters_last = it + 1;
      s->delta_last = s->hdelta[0];
      HIPCHK(launch_finish(a, s->stream));
      break;
    }
    ++it;
  }
  s->iters_max = std::max(s->iters_max, s->iters_last);
  s->lu_step = false;
  return corrector<T>(s, nullptr);
}

// The predictor's solve with the sine transforms on the matrix cores (FP32 flow only):
// right-hand side rows -> (rows) . S -> S . (columns) with the spectral solve -> S . for s and
// gamma, leaving the same row-spectral arrays as the transform kernels (work, workg).
template <typename T>
ib_status gemm_solve(ib_solver* s, RhsArgs<T>& a, double alpha, bool has_ring) {
  if constexpr (sizeof(T) != 4) {
    return IB_ERR_STATE;
  } else {
    const int n = s->n, P = s->pitch;
    a.out = static_cast<T*>(s->work2);
    {
      TimeScope ts(s, IB_K_RHS_ROWDST);
      HIPCHK(launch_rhs_rowdst<T>(a, s->tw, s->stream, 0));
      GemmArgs g{};
      g.shi = static_cast<const __bf16*>(s->shi);
      g.slo = static_cast<const __bf16*>(s->slo);
      g.ps = s->kpad;
      g.nv = n - 1;
      g.kpad = s->kpad;
      g.x = static_cast<const float*>(s->work2);
      g.px = P;
      g.c = static_cast<float*>(s->work);
      g.pc = P;
      g.tn = s->gemm_tn;
      HIPCHK(launch_dst_gemm(g, 1, s->stream));
    }
    TimeScope ts(s, IB_K_COL_SOLVE);
    GemmArgs g{};
    g.shi = static_cast<const __bf16*>(s->shi);
    g.slo = static_cast<const __bf16*>(s->slo);
    g.ps = s->kpad;
    g.nv = n - 1;
    g.kpad = s->kpad;
    g.x = static_cast<const float*>(s->work);
    g.px = P;
    g.c = s->ys;
    g.pc = P;
    g.c2 = s->yg;
    g.pc2 = P;
    g.lam = static_cast<const float*>(s->lam);
    g.alpha = (float)alpha;
    g.scale = (float)(4.0 / ((double)n * n));
    g.lift = has_ring ? static_cast<const float*>(s->lift) : nullptr;
    g.sinv = s->sinv;
    g.tn = s->gemm_tn;
    HIPCHK(launch_dst_gemm(g, 0, s->stream));
    GemmArgs h{};
    h.shi = g.shi;
    h.slo = g.slo;
    h.ps = g.ps;
    h.nv = g.nv;
    h.kpad = g.kpad;
    h.px = h.pc = P;
    h.tn = s->gemm_tn;
    h.x = s->ys;
    h.c = static_cast<float*>(s->work);
    HIPCHK(launch_dst_gemm(h, 0, s->stream));
    h.x = s->yg;
    h.c = static_cast<float*>(s->workg);
    HIPCHK(launch_dst_gemm(h, 0, s->stream));
    return IB_OK;
  }
}

// Enqueue one step (Algorithm 2): for every level, coarse to fine, the ring from the coarser
// level, the explicit right-hand side and the predictor solve; on level 0 with bodies the
// FSI iterations and the corrector; then each level's inverse row transform into its state.
// With `ahead` (moving bodies) the FSI iterations, the corrector and level 0's final
// transform are launched ahead under the device gates and nothing here waits for the GPU,
// so the launches can be recorded as a graph; otherwise the host tests every FSI iteration.
// Host state that changes per step (ring buffer alternation, step count) is left alone.
// One level of the predictor: its new ring from the next coarser level, the right-hand side
// and the transforms into the spectral scratch (work, workg), then its inverse row transform
// into the state; on level 0 with bodies the s* rows and the FSI part come first.  first:
// the step has no history yet.
template <typename T>
ib_status enqueue_level(ib_solver* s, int g, bool ahead, int K, bool first, void* work,
                        void* workg, bool ring_made = false) {
  const int n = s->n, ny = s->ny, G = (int)s->lv.size(), P = s->pitch;
  const bool bodies = !s->bodies.empty();
  {
    LevelState& L = s->lv[g];
    const bool has_ring = g < G - 1;
    const int nxt = 1 - L.gcur;
    // ring_made: the side stream already made this level's ring (level 1 after the levels
    // launched ahead), with its edge transforms in lift_l1
    void* lift = ring_made ? s->lift_l1 : s->lift;
    if (has_ring && !ring_made) {
      TimeScope ts(s, IB_K_RING);
      HIPCHK(launch_ring_dst<T>(static_cast<T*>(s->lv[g + 1].s), P,
                                static_cast<T*>(s->lv[g + 1].g), P, n, ny,
                                static_cast<T*>(L.sring), static_cast<T*>(L.gring[nxt]), s->tw,
                                twy_of(s), static_cast<T*>(s->lift), s->stream));
    }
    RhsArgs<T> a{};
    a.s = static_cast<T*>(L.s);
    a.g = static_cast<T*>(L.g);
    a.gf = g > 0 ? static_cast<T*>(s->lv[g - 1].g) : nullptr;
    a.gring = static_cast<T*>(L.gring[L.gcur]);
    a.gring_new = has_ring ? static_cast<T*>(L.gring[nxt]) : nullptr;
    a.hist_in = first ? nullptr : static_cast<T*>(L.hist);
    a.hist_out = static_cast<T*>(L.hist);
    a.out = static_cast<T*>(work);
    a.n = n;
    a.ny = ny;
    a.ps = a.pg = a.pgf = a.ph = a.po = P;
    a.alpha = (T)L.alpha;
    a.dt = (T)s->cfg.dt;
    a.ux = (T)(s->cfg.u_inf[0] * L.h);
    a.uy = (T)(s->cfg.u_inf[1] * L.h);
    a.cn = (T)(-1.0 / (2.0 * L.h * L.h));
    a.var = s->tune.rhs;
    ib_status st = IB_OK;
    if (s->gemm) {
      a.var = 0;
      st = gemm_solve(s, a, L.alpha, has_ring);
    } else {
      {
        TimeScope ts(s, IB_K_RHS_ROWDST);
        HIPCHK(launch_rhs_rowdst<T>(a, s->tw, s->stream));
      }
      TimeScope ts(s, IB_K_COL_SOLVE, true);
      st = solve_into<T>(s, work, L.alpha, 4.0 / ((double)n * ny), 1, ny - 1, s->tw, s->lam,
                         workg, has_ring ? lift : nullptr, s->tune.col, ts.b, ts.e);
    }
    if (st) return st;
    RowArgs<T> r{};
    r.in = static_cast<T*>(work);
    r.pi = r.po = P;
    const T* ring = has_ring ? static_cast<T*>(L.sring) : nullptr;
    const int* gate = nullptr;
    if (g == 0 && bodies) {
      // s* on the rows the body operators can reach
      r.out = static_cast<T*>(s->sstar);
      r.r0 = std::max(1, s->blo - 3);
      r.r1 = std::min(n - 1, s->bhi + 3);
      // the same launch clears the step's control block (flags, gates, counters)
      r.reset = s->flags;
      r.nreset = FsiCtl::INTS;
      {
        TimeScope ts(s, IB_K_ROW_IDST);
        HIPCHK(launch_row_idst<T>(r, n, 1, s->tw, ring, 0, s->stream));
      }
      r.reset = nullptr;
      if (ahead) {
        st = fsi_launch_ahead<T>(s, K);
        gate = s->gate;
        if (!st && s->ctl_early) {
          // the control block is final after the iterations: the host can read it and
          // queue the next step while the (gated) corrector's inverse row transform still
          // runs (copied earlier, before the corrector, the host's next launches slowed
          // the step: 0.380 against 0.375 ms)
          HIPCHK(hipMemcpyAsync(s->hctl, s->ctl, FsiCtl::BYTES, hipMemcpyDeviceToHost, s->stream));
          HIPCHK(hipEventRecord(s->ctl_ready, s->stream));
        }
      } else {
        st = fsi_host<T>(s, 0);
      }
      if (st) return st;
    }
    r.out = static_cast<T*>(L.s);
    r.r0 = 1;
    r.r1 = ny - 1;
    r.ny = ny;
    r.in2 = static_cast<T*>(workg);
    r.out2 = static_cast<T*>(L.g);
    r.var = s->tune.idst;
    r.gate = gate;
    {
      TimeScope ts(s, IB_K_ROW_IDST);
      HIPCHK(launch_row_idst<T>(r, n, 1, s->tw, ring, 1, s->stream));
    }
  }
  return IB_OK;
}

// The next step's levels G-1 .. 2 on the side stream, after this step's level 1 (l1_done,
// recorded on the solver's stream).  With three or more levels they read only their own states,
// the next finer level's circulation (coarsification on read) and rings made from the
// next coarser level, all final once this step's level 1 is: level 1 is never corrected, and
// nothing of this step after level 1 reads a level >= 2.  So they run concurrently with
// this step's level 0, FSI part and corrector, with spectral scratch and ring transforms of
// their own, and give the same results bit for bit.  Their ring parity is the next step's
// (the end of a step flips it).  Level 1's ring for the next step follows them there.
template <typename T>
ib_status launch_side_levels(ib_solver* s) {
  const int G = (int)s->lv.size();
  HIPCHK(hipStreamWaitEvent(s->side, s->l1_done, 0));
  struct Swap {
    ib_solver* s;
    hipStream_t stream;
    void* lift;
    Swap(ib_solver* s_) : s(s_), stream(s_->stream), lift(s_->lift) {
      s->stream = s->side;
      s->lift = s->lift_pre;
      for (int g = 2; g < (int)s->lv.size() - 1; ++g) s->lv[g].gcur ^= 1;
    }
    ~Swap() {
      s->stream = stream;
      s->lift = lift;
      for (int g = 2; g < (int)s->lv.size() - 1; ++g) s->lv[g].gcur ^= 1;
    }
  };
  {
    Swap sw(s);
    for (int g = G - 1; g >= 2; --g) {
      ib_status st = enqueue_level<T>(s, g, false, 0, false, s->work_pre, s->workg_pre);
      if (st) return st;
    }
  }
  // Level 1's ring for the next step, from level 2's new state: nothing of this step reads
  // level 1's ring after l1_done, and its new circulation ring goes to the buffer that this
  // step's level 1 read as the old one (the parity flips at the end of the step).
  {
    LevelState& L1 = s->lv[1];
    HIPCHK(launch_ring_dst<T>(static_cast<T*>(s->lv[2].s), s->pitch,
                              static_cast<T*>(s->lv[2].g), s->pitch, s->n, s->ny,
                              static_cast<T*>(L1.sring), static_cast<T*>(L1.gring[L1.gcur]),
                              s->tw, twy_of(s), static_cast<T*>(s->lift_l1), s->side));
  }
  HIPCHK(hipEventRecord(s->side_done, s->side));
  s->side_ahead = true;
  return IB_OK;
}

// A step's levels from gtop (the coarsest, G - 1, unless it was launched ahead) to 0; with
// side_next, the next step's levels >= 2 go to the side stream, waiting there for this
// step's level 1.  They are enqueued after level 0 and the FSI part, so that the host has
// queued this step's long dependent chain first and the side stream's kernels run beside it.
template <typename T>
ib_status enqueue_step(ib_solver* s, bool ahead, int K, int gtop = -1, bool side_next = false) {
  const int G = (int)s->lv.size();
  int g0 = gtop < 0 ? G - 1 : gtop;
  bool side_ran = false;
  if (s->side_ahead) {
    // levels G-1 .. 2 of this step, and level 1's ring, ran on the side stream
    HIPCHK(hipStreamWaitEvent(s->stream, s->side_done, 0));
    s->side_ahead = false;
    side_ran = true;
    g0 = 1;
  }
  for (int g = g0; g >= 0; --g) {
    ib_status st = enqueue_level<T>(s, g, ahead, K, s->first, s->work, s->workg,
                                    side_ran && g == 1);
    if (st) return st;
    if (g == 1 && side_next) {
      if (!s->side) {
        // created at first use: solvers that never step alone add no stream (the runtime
        // maps every stream of the process onto a few hardware queues)
        HIPCHK(hipStreamCreateWithFlags(&s->side, hipStreamNonBlocking));
        HIPCHK(hipEventCreateWithFlags(&s->l1_done, hipEventDisableTiming));
        HIPCHK(hipEventCreateWithFlags(&s->side_done, hipEventDisableTiming));
      }
      HIPCHK(hipEventRecord(s->l1_done, s->stream));
    }
  }
  if (side_next) return launch_side_levels<T>(s);
  return IB_OK;
}

// Level 0's inverse row transform into its state (the last launch of a step), after the
// FSI part was finished on the host.
template <typename T>
ib_status final_transform_level0(ib_solver* s) {
  const int n = s->n, G = (int)s->lv.size(), P = s->pitch;
  LevelState& L = s->lv[0];
  RowArgs<T> r{};
  r.in = static_cast<T*>(s->work);
  r.pi = r.po = P;
  r.out = static_cast<T*>(L.s);
  r.r0 = 1;
  r.r1 = s->ny - 1;
  r.ny = s->ny;
  r.in2 = static_cast<T*>(s->workg);
  r.out2 = static_cast<T*>(L.g);
  r.var = s->tune.idst;
  const T* ring = G > 1 ? static_cast<T*>(L.sring) : nullptr;
  TimeScope ts(s, IB_K_ROW_IDST);
  HIPCHK(launch_row_idst<T>(r, n, 1, s->tw, ring, 1, s->stream));
  return IB_OK;
}

void destroy_graphs(ib_solver* s) {
  for (auto& row : s->step_graphs)
    for (auto& g : row) {
      if (g.exec) (void)hipGraphExecDestroy(g.exec);
      g = StepGraph{};
    }
}

// How the next step runs: FSI iterations launched ahead (and how many), and whether it
// is replayed from a recorded graph (for which ring-buffer alternation).
struct StepPlan {
  bool ahead = false, use_graph = false;
  int K = 0, parity = 0;
  bool refresh0 = false;  // the first FSI iteration refreshes the approximate inverse
};

StepPlan plan_step(const ib_solver* s) {
  StepPlan p;
  const bool bodies = !s->bodies.empty();
  p.ahead = bodies && fsi_ahead(s);
  const bool sync_free = !bodies || s->stationary || p.ahead;
  p.K = p.ahead ? fsi_ahead_count(s) : 0;
  // (the legacy null stream cannot be recorded)
  p.use_graph = s->graphs && s->fsi_ahead && sync_free && !s->first && !s->timing &&
                s->stream != nullptr;
  p.parity = s->lv.size() > 1 ? s->lv[0].gcur : 0;
  p.refresh0 = refresh_at(s, 0);
  return p;
}

const StepGraph* find_graph(const ib_solver* s, const StepPlan& p) {
  for (const StepGraph& g : s->step_graphs[p.parity])
    if (g.exec && g.K == p.K && g.refresh0 == p.refresh0) return &g;
  return nullptr;
}

bool needs_record(const ib_solver* s, const StepPlan& p) {
  return p.use_graph && find_graph(s, p) == nullptr;
}

// Record the step's launches as a graph (nothing runs).  The caller holds the library's
// exclusive HIP lock: on this runtime another thread's synchronising calls fail while a
// stream records.  A failed recording turns graphs off for this solver.
template <typename T>
ib_status record_step(ib_solver* s, const StepPlan& p) {
  int& next = s->graph_next[p.parity];
  StepGraph& sg = s->step_graphs[p.parity][next];
  next = (next + 1) % ib_solver::GRAPH_SLOTS;
  if (sg.exec) (void)hipGraphExecDestroy(sg.exec);
  sg = StepGraph{};
  hipGraph_t graph = nullptr;
  hipError_t e = hipStreamBeginCapture(s->stream, hipStreamCaptureModeRelaxed);
  if (e == hipSuccess) {
    ib_status st = enqueue_step<T>(s, p.ahead, p.K);
    e = hipStreamEndCapture(s->stream, &graph);
    if (st) {
      if (graph) (void)hipGraphDestroy(graph);
      return st;
    }
  }
  if (e == hipSuccess) {
    e = hipGraphInstantiate(&sg.exec, graph, nullptr, nullptr, 0);
    if (e != hipSuccess) sg = StepGraph{};
  }
  if (graph) (void)hipGraphDestroy(graph);
  if (e == hipSuccess) {
    sg.K = p.K;
    sg.refresh0 = p.refresh0;
    s->graph_captures++;
  } else {
    (void)hipGetLastError();
    s->graphs = false;
    s->graph_failures++;
  }
  return IB_OK;
}

// Whether the next step's coarsest level can be launched while the host waits for this
// step's convergence tests: it reads only its own level and the next finer level's
// circulation (coarsification on read), both final before this step's FSI part when there
// are three or more levels (with two, the finer level is level 0, whose final transform
// waits for convergence and may still be redone on the host), and it has spectral scratch
// of its own, so nothing the host may still add to this step touches it.
bool can_launch_top_ahead(const ib_solver* s) {
  return s->lv.size() >= 3 && s->work_pre != nullptr && !s->gemm && !s->timing && !s->graphs &&
         s->ahead_mode == 1 && g_stepping.load(std::memory_order_relaxed) == 1;
}

// Whether the next step's levels >= 2 can run on the side stream (launch_side_levels).
bool can_launch_side(const ib_solver* s) {
  return s->lv.size() >= 3 && s->work_pre != nullptr && s->lift_pre != nullptr && !s->gemm &&
         !s->timing && !s->graphs && s->ahead_mode == 2 &&
         g_stepping.load(std::memory_order_relaxed) == 1;
}

// pre_next: the caller takes another step right after this one (its coarsest level may be
// launched ahead).
template <typename T>
ib_status do_step(ib_solver* s, const StepPlan& p, bool pre_next = false) {
  const int G = (int)s->lv.size();
  if (s->nmov) {
    ib_status pst = update_poses(s, (s->step + 1) * s->cfg.dt);  // constraint at t_{n+1}
    if (pst) return pst;
  }
  ib_status st = IB_OK;
  const StepGraph* sg = p.use_graph && s->graphs ? find_graph(s, p) : nullptr;
  if (sg) {
    HIPCHK(hipGraphLaunch(sg->exec, s->stream));
    s->graph_launches++;
  } else {
    // without the coarsest level launched during the host wait (IB_OPT_TOP_AHEAD = 1), the
    // control block is copied as soon as the FSI iterations are queued
    s->ctl_early = p.ahead && s->ahead_mode != 1;
    if (s->ctl_early && !s->ctl_ready)
      HIPCHK(hipEventCreateWithFlags(&s->ctl_ready, hipEventDisableTiming));
    st = enqueue_step<T>(s, p.ahead, p.K, s->top_ahead ? G - 2 : -1,
                         pre_next && can_launch_side(s));
    s->ctl_early = false;
    if (st) return st;
  }
  s->top_ahead = false;
  if (p.ahead) {
    if (!sg && s->ahead_mode != 1) {
      // copied after the corrector's column solve (enqueue_level); its last transform may still run
      HIPCHK(hipEventSynchronize(s->ctl_ready));
    } else {
      HIPCHK(hipMemcpyAsync(s->hctl, s->ctl, FsiCtl::BYTES, hipMemcpyDeviceToHost, s->stream));
      if (pre_next && can_launch_top_ahead(s) && !sg) {
        if (!s->ctl_ready) HIPCHK(hipEventCreateWithFlags(&s->ctl_ready, hipEventDisableTiming));
        HIPCHK(hipEventRecord(s->ctl_ready, s->stream));
        st = enqueue_level<T>(s, G - 1, false, 0, false, s->work_pre, s->workg_pre);
        if (st) return st;
        s->top_ahead = true;
        HIPCHK(hipEventSynchronize(s->ctl_ready));
      } else {
        HIPCHK(hipStreamSynchronize(s->stream));
      }
    }
    int resume = -1;
    st = fsi_after_ahead(s, &resume);
    if (st) return st;
    if (resume >= 0) {
      // the launched iterations did not suffice: finish the FSI part on the host, then
      // level 0's final transform (skipped on the device)
      s->fsi_resumes++;
      st = fsi_host<T>(s, resume);
      if (st) return st;
      st = final_transform_level0<T>(s);
      if (st) return st;
    }
  }
  for (int g = 0; g < G - 1; ++g) s->lv[g].gcur = 1 - s->lv[g].gcur;
  s->first = false;
  s->step++;
  return IB_OK;
}

// BF16 split of the sine matrix S_jk = sin(pi (j+1)(k+1) / n), zero padded to kpad, plus
// sin(pi k / n), k <= n, and the two spectral work arrays of the matrix-core transforms.
uint16_t bf16_bits(float f) {
  uint32_t u;
  std::memcpy(&u, &f, 4);
  u += 0x7FFFu + ((u >> 16) & 1u);  // round to nearest even (finite inputs)
  return (uint16_t)(u >> 16);
}
float bf16_value(uint16_t b) {
  const uint32_t u = (uint32_t)b << 16;
  float f;
  std::memcpy(&f, &u, 4);
  return f;
}
ib_status make_gemm_tables(ib_solver* s) {
  const int n = s->n, nv = n - 1;
  s->kpad = round_up(nv, 64);
  const int kp = s->kpad;
  std::vector<uint16_t> hi((size_t)kp * kp, 0), lo((size_t)kp * kp, 0);
  for (int j = 0; j < nv; ++j)
    for (int k = 0; k < nv; ++k) {
      const float v = (float)std::sin(M_PI * (double)(j + 1) * (double)(k + 1) / n);
      const uint16_t h = bf16_bits(v);
      hi[(size_t)j * kp + k] = h;
      lo[(size_t)j * kp + k] = bf16_bits(v - bf16_value(h));
    }
  std::vector<float> sv(n + 1);
  for (int k = 0; k <= n; ++k) sv[k] = (float)std::sin(M_PI * k / n);
  s->shi = dalloc(s, hi.size() * 2);
  s->slo = dalloc(s, lo.size() * 2);
  s->sinv = static_cast<float*>(dalloc(s, sv.size() * 4));
  s->ys = static_cast<float*>(dalloc(s, (size_t)nv * s->pitch * 4));
  s->yg = static_cast<float*>(dalloc(s, (size_t)nv * s->pitch * 4));
  if (!s->shi || !s->slo || !s->sinv || !s->ys || !s->yg) return IB_ERR_OOM;
  HIPCHK(hipMemcpy(s->shi, hi.data(), hi.size() * 2, hipMemcpyHostToDevice));
  HIPCHK(hipMemcpy(s->slo, lo.data(), lo.size() * 2, hipMemcpyHostToDevice));
  HIPCHK(hipMemcpy(s->sinv, sv.data(), sv.size() * 4, hipMemcpyHostToDevice));
  return IB_OK;
}

// Measured stage depth of the sine-transform products (64 or 128 values of k per stage): the
// column product (the plain form of the three S . products of a level) timed with each on the
// spectral scratch arrays (their contents do not matter for the time), the faster kept.
ib_status tune_gemm(ib_solver* s) {
  s->gemm_tn = 64;
  if (s->kpad % 128 != 0) return IB_OK;
  GemmArgs g{};
  g.shi = static_cast<const __bf16*>(s->shi);
  g.slo = static_cast<const __bf16*>(s->slo);
  g.ps = s->kpad;
  g.nv = s->n - 1;
  g.kpad = s->kpad;
  g.x = static_cast<const float*>(s->work);
  g.px = g.pc = s->pitch;
  g.c = static_cast<float*>(s->workg);
  hipEvent_t e0 = nullptr, e1 = nullptr;
  hipError_t e = hipEventCreate(&e0);
  if (e == hipSuccess) e = hipEventCreate(&e1);
  float best = 0.0f;
  for (int bk : {64, 128}) {
    if (e != hipSuccess) break;
    g.tn = bk;
    for (int r = 0; r < 2 && e == hipSuccess; ++r) e = launch_dst_gemm(g, 0, s->stream);
    if (e == hipSuccess) e = hipEventRecord(e0, s->stream);
    for (int r = 0; r < 5 && e == hipSuccess; ++r) e = launch_dst_gemm(g, 0, s->stream);
    if (e == hipSuccess) e = hipEventRecord(e1, s->stream);
    if (e == hipSuccess) e = hipEventSynchronize(e1);
    float ms = 0.0f;
    if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
    if (e == hipSuccess && (bk == 64 || ms < best)) {
      best = ms;
      s->gemm_tn = bk;
    }
  }
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  if (e != hipSuccess) return hip_fail(s, e, "sine-transform product timing");
  return IB_OK;
}

// Device state of the levels (allocated by ib_prepare, so that creating a solver costs
// no device memory and a scheduler can admit it later).
ib_status alloc_state(ib_solver* s) {
  const size_t full = (size_t)(s->ny + 1) * s->pitch * s->es;
  const size_t inner = (size_t)(s->ny - 1) * s->pitch * s->es;
  const size_t ring = (size_t)ring_len(s->n, s->ny) * s->es;
  const size_t lift = (size_t)(2 * (s->n - 1) + 2 * (s->ny - 1)) * s->es;
  for (auto& L : s->lv) {
    L.s = dalloc(s, full);
    L.g = dalloc(s, inner);
    L.hist = dalloc(s, inner);
    L.sring = dalloc(s, ring);
    L.gring[0] = dalloc(s, ring);
    L.gring[1] = dalloc(s, ring);
    if (!L.s || !L.g || !L.hist || !L.sring || !L.gring[0] || !L.gring[1]) return IB_ERR_OOM;
  }
  s->work = dalloc(s, inner);
  s->workg = dalloc(s, inner);
  s->work2 = dalloc(s, inner);
  s->work_pre = s->workg_pre = s->lift_pre = s->lift_l1 = nullptr;
  s->top_ahead = s->side_ahead = false;
  if (s->lv.size() >= 3 && !s->gemm) {
    s->work_pre = dalloc(s, inner);
    s->workg_pre = dalloc(s, inner);
    s->lift_pre = dalloc(s, lift);
    s->lift_l1 = dalloc(s, lift);
    if (!s->work_pre || !s->workg_pre || !s->lift_pre || !s->lift_l1) return IB_ERR_OOM;
  }
  s->lift = dalloc(s, lift);
  s->sstar = dalloc(s, full);
  if (!s->work || !s->workg || !s->work2 || !s->sstar || !s->lift) return IB_ERR_OOM;
  ib_status st = s->fp64 ? make_tables<double>(s, s->n, &s->tw, &s->lam)
                         : make_tables<float>(s, s->n, &s->tw, &s->lam);
  if (st == IB_OK) st = make_tables<double>(s, s->n, &s->tw64, &s->lam64);
  if (st == IB_OK && s->ny != s->n) st = s->fp64 ? make_rect_tables<double>(s) : make_rect_tables<float>(s);
  if (st == IB_OK && s->gemm) st = make_gemm_tables(s);
  if (st == IB_OK && s->gemm) st = tune_gemm(s);
  if (st) return st;
  for (auto& L : s->lv) {
    HIPCHK(hipMemsetAsync(L.s, 0, full, s->stream));
    HIPCHK(hipMemsetAsync(L.hist, 0, inner, s->stream));
    HIPCHK(hipMemsetAsync(L.g, 0, inner, s->stream));
    HIPCHK(hipMemsetAsync(L.sring, 0, ring, s->stream));
    HIPCHK(hipMemsetAsync(L.gring[0], 0, ring, s->stream));
    HIPCHK(hipMemsetAsync(L.gring[1], 0, ring, s->stream));
  }
  HIPCHK(hipMemsetAsync(s->work2, 0, inner, s->stream));
  HIPCHK(hipMemsetAsync(s->sstar, 0, full, s->stream));
  s->allocated = true;
  return IB_OK;
}

ib_status check(ib_solver* s) {
  if (!s) return IB_ERR_ARG;
  return IB_OK;
}

// ------------------------------------------------------------------ batches
//
// A batch steps many solvers together: every launch of a step covers all members that
// need it (one launch per grid size for the flow kernels, one for all members for the
// FSI kernels), with each member's arguments in a table that is built on the host and
// moved to the device with one copy before the step's first launch.  Each member keeps
// its own state, scratch and control block, and every kernel computes exactly what it
// computes for the member alone.

// One step's launch tables (host bytes, 256-byte aligned entries) and the launches that
// read them, in stream order.
struct BatchPlan {
  std::vector<char> tab;
  std::vector<std::function<hipError_t(const char*)>> launches;

  template <class J>
  size_t put(const std::vector<J>& v) {
    const size_t off = (tab.size() + 255) & ~size_t(255);
    tab.resize(off + v.size() * sizeof(J));
    std::memcpy(tab.data() + off, v.data(), v.size() * sizeof(J));
    return off;
  }
  // f(device table, count) issues the launch
  template <class J, class F>
  void add(const std::vector<J>& v, F f) {
    if (v.empty()) return;
    const size_t off = put(v);
    const int count = (int)v.size();
    launches.push_back(
        [off, count, f](const char* d) { return f(reinterpret_cast<const J*>(d + off), count); });
  }
};

}  // namespace

struct ib_batch {
  std::vector<ib_solver*> mem;
  hipStream_t stream = nullptr;
  bool fp64 = false;
  // launch tables: two slots (alternate steps), pinned host staging and device copies
  char* hbuf[2] = {nullptr, nullptr};
  char* dbuf[2] = {nullptr, nullptr};
  hipEvent_t copied[2] = {nullptr, nullptr};
  hipEvent_t ctl_ready = nullptr;  // the members' control blocks of this step are on the host
  size_t cap = 0;
  int slot = 0;
  // gathered control blocks of the members iterating on the device, and their mirror
  int* dctl = nullptr;
  int* hctl = nullptr;
  int ctl_cap = 0;
  int64_t steps = 0, member_steps_batched = 0, member_steps_alone = 0, launches = 0,
          resumes = 0;
  std::string last_error;
};

namespace {

ib_status batch_hip(ib_batch* b, hipError_t e, const char* what) {
  b->last_error = std::string(what) + ": " + hipGetErrorString(e);
  return IB_ERR_HIP;
}

#define BCHK(expr)                                        \
  do {                                                    \
    hipError_t e_ = (expr);                               \
    if (e_ != hipSuccess) return batch_hip(b, e_, #expr); \
  } while (0)

void batch_free_buffers(ib_batch* b) {
  for (int k = 0; k < 2; ++k) {
    if (b->hbuf[k]) (void)hipHostFree(b->hbuf[k]);
    if (b->dbuf[k]) (void)hipFree(b->dbuf[k]);
    b->hbuf[k] = b->dbuf[k] = nullptr;
  }
  b->cap = 0;
}

ib_status batch_reserve(ib_batch* b, size_t bytes, int nctl) {
  if (bytes > b->cap) {
    BCHK(hipStreamSynchronize(b->stream));  // nothing may still read the old tables
    batch_free_buffers(b);
    const size_t cap = std::max<size_t>(bytes * 2, 64 * 1024);
    for (int k = 0; k < 2; ++k) {
      if (hipHostMalloc(reinterpret_cast<void**>(&b->hbuf[k]), cap, 0) != hipSuccess ||
          hipMalloc(reinterpret_cast<void**>(&b->dbuf[k]), cap) != hipSuccess) {
        batch_free_buffers(b);
        b->last_error = "launch tables of the batch";
        return IB_ERR_OOM;
      }
    }
    b->cap = cap;
  }
  if (nctl > b->ctl_cap) {
    BCHK(hipStreamSynchronize(b->stream));
    if (b->dctl) (void)hipFree(b->dctl);
    if (b->hctl) (void)hipHostFree(b->hctl);
    b->dctl = nullptr;
    b->hctl = nullptr;
    b->ctl_cap = 0;
    const size_t bytes_ctl = (size_t)nctl * FsiCtl::BYTES;
    if (hipMalloc(reinterpret_cast<void**>(&b->dctl), bytes_ctl) != hipSuccess ||
        hipHostMalloc(reinterpret_cast<void**>(&b->hctl), bytes_ctl, 0) != hipSuccess) {
      b->last_error = "control blocks of the batch";
      return IB_ERR_OOM;
    }
    b->ctl_cap = nctl;
  }
  return IB_OK;
}

// Members whose next step runs alone: their first step (no history yet), a step whose
// Schur inverse must first be built (host-driven LU) or whose FSI part is host-driven, and
// members with the matrix-core transforms or kernel timing on.
bool steps_alone(const ib_solver* s) {
  return s->first || s->gemm || s->timing ||
         (!s->bodies.empty() && !s->stationary && !fsi_ahead(s));
}

// Members of one flow launch: the same grid size and kernel configurations.
struct FlowGroup {
  int n = 0, vr = 0, vc = 0, vi = 0;
  std::vector<ib_solver*> m;
};

template <typename T>
ib_status batch_step(ib_batch* b) {
  // members that step alone this time (host-driven path, on the batch's stream)
  std::vector<ib_solver*> ready;
  for (ib_solver* s : b->mem) {
    if (!steps_alone(s)) {
      ready.push_back(s);
      continue;
    }
    StepPlan p = plan_step(s);
    p.use_graph = false;
    ib_status st = do_step<T>(s, p);
    if (st) {
      s->failed = true;
      b->last_error = s->last_error;
      return st;
    }
    b->member_steps_alone++;
  }
  if (ready.empty()) return IB_OK;
  for (ib_solver* s : ready) {
    if (!s->nmov) continue;
    ib_status st = update_poses(s, (s->step + 1) * s->cfg.dt);  // constraint at t_{n+1}
    if (st) {
      s->failed = true;
      b->last_error = s->last_error;
      return st;
    }
  }
  std::vector<FlowGroup> groups;
  std::vector<ib_solver*> bodied, iter, stat;
  int gmax = 0, K = 0;
  for (ib_solver* s : ready) {
    FlowGroup* grp = nullptr;
    for (auto& q : groups)
      if (q.n == s->n && q.vr == s->tune.rhs && q.vc == s->tune.col && q.vi == s->tune.idst)
        grp = &q;
    if (!grp) {
      groups.push_back(FlowGroup{s->n, s->tune.rhs, s->tune.col, s->tune.idst, {}});
      grp = &groups.back();
    }
    grp->m.push_back(s);
    gmax = std::max(gmax, (int)s->lv.size());
    if (s->bodies.empty()) continue;
    bodied.push_back(s);
    if (s->stationary) {
      stat.push_back(s);
    } else {
      iter.push_back(s);
      K = std::max(K, fsi_ahead_count(s));
    }
  }
  BatchPlan pl;
  hipStream_t st = b->stream;
  auto gate_of = [](const ib_solver* s) -> const int* { return s->stationary ? nullptr : s->gate; };

  // ---- predictor, coarse to fine (levels counted from each member's finest)
  for (int g = gmax - 1; g >= 0; --g) {
    for (auto& q : groups) {
      std::vector<RingJob<T>> rings;
      std::vector<RhsArgs<T>> rhs;
      std::vector<ColArgs<T>> cols;
      std::vector<IdstJob<T>> star, fin;
      int star_rows = 0;
      const void* tw = q.m[0]->tw;
      const void* lam = q.m[0]->lam;
      for (ib_solver* s : q.m) {
        const int G = (int)s->lv.size(), n = s->n, P = s->pitch;
        if (g >= G) continue;
        LevelState& L = s->lv[g];
        const bool has_ring = g < G - 1;
        const int nxt = 1 - L.gcur;
        if (has_ring)
          rings.push_back(RingJob<T>{static_cast<const T*>(s->lv[g + 1].s), P,
                                     static_cast<const T*>(s->lv[g + 1].g), P,
                                     static_cast<T*>(L.sring), static_cast<T*>(L.gring[nxt]),
                                     static_cast<T*>(s->lift)});
        RhsArgs<T> a{};
        a.s = static_cast<T*>(L.s);
        a.g = static_cast<T*>(L.g);
        a.gf = g > 0 ? static_cast<T*>(s->lv[g - 1].g) : nullptr;
        a.gring = static_cast<T*>(L.gring[L.gcur]);
        a.gring_new = has_ring ? static_cast<T*>(L.gring[nxt]) : nullptr;
        a.hist_in = static_cast<T*>(L.hist);
        a.hist_out = static_cast<T*>(L.hist);
        a.out = static_cast<T*>(s->work);
        a.n = n;
        a.ps = a.pg = a.pgf = a.ph = a.po = P;
        a.alpha = (T)L.alpha;
        a.dt = (T)s->cfg.dt;
        a.ux = (T)(s->cfg.u_inf[0] * L.h);
        a.uy = (T)(s->cfg.u_inf[1] * L.h);
        a.cn = (T)(-1.0 / (2.0 * L.h * L.h));
        a.var = s->tune.rhs;
        rhs.push_back(a);
        ColArgs<T> c{};
        c.var = s->tune.col;
        c.in = static_cast<T*>(s->work);
        c.out = static_cast<T*>(s->work);
        c.out2 = static_cast<T*>(s->workg);
        c.lift = has_ring ? static_cast<const T*>(s->lift) : nullptr;
        c.pi = c.po = P;
        c.r0 = 1;
        c.r1 = n - 1;
        c.alpha = (T)L.alpha;
        c.scale = (T)(4.0 / ((double)n * n));
        c.w0 = 1;
        c.w1 = n - 1;
        cols.push_back(c);
        const T* ring = has_ring ? static_cast<T*>(L.sring) : nullptr;
        if (g == 0 && !s->bodies.empty()) {
          RowArgs<T> r{};
          r.in = static_cast<T*>(s->work);
          r.pi = r.po = P;
          r.out = static_cast<T*>(s->sstar);
          r.r0 = std::max(1, s->blo - 3);
          r.r1 = std::min(n - 1, s->bhi + 3);
          star.push_back(IdstJob<T>{r, ring, 0});
          star_rows = std::max(star_rows, r.r1 - r.r0 + 1);
        }
        if (g > 0) {
          RowArgs<T> r{};
          r.in = static_cast<T*>(s->work);
          r.pi = r.po = P;
          r.out = static_cast<T*>(L.s);
          r.r0 = 1;
          r.r1 = n - 1;
          r.in2 = static_cast<T*>(s->workg);
          r.out2 = static_cast<T*>(L.g);
          r.var = s->tune.idst;
          fin.push_back(IdstJob<T>{r, ring, 1});
        }
      }
      const int n = q.n, vr = q.vr, vc = q.vc, vi = q.vi;
      pl.add(rings, [=](const RingJob<T>* d, int c) { return launch_ring_multi<T>(d, c, n, tw, st); });
      pl.add(rhs, [=](const RhsArgs<T>* d, int c) {
        return launch_rhs_rowdst_multi<T>(d, c, n, vr, tw, st);
      });
      pl.add(cols, [=](const ColArgs<T>* d, int c) {
        return launch_col_solve_multi<T>(d, c, n, vc, tw, lam, st);
      });
      pl.add(star, [=](const IdstJob<T>* d, int c) {
        return launch_row_idst_multi<T>(d, c, n, star_rows, 0, 0, tw, st);
      });
      pl.add(fin, [=](const IdstJob<T>* d, int c) {
        return launch_row_idst_multi<T>(d, c, n, n - 1, 1, vi, tw, st);
      });
    }
  }

  // ---- FSI part (Algorithm 2's loop) for every member with bodies
  std::vector<int*> ctls;
  for (ib_solver* s : bodied) ctls.push_back(s->flags);
  pl.add(ctls, [=](int* const* d, int c) { return launch_step_reset_multi(d, c, st); });
  {
    // stationary bodies: f = M^{-1} rhs
    std::vector<FsiArgs> ops;
    std::vector<MatvecJob> mv;
    int max_pts = 0, max_nf = 0;
    for (ib_solver* s : stat) {
      FsiArgs a = s->fa;
      a.iter = 0;
      ops.push_back(a);
      mv.push_back(MatvecJob{s->Minv, a.pm, s->rhs, s->f, s->nf});
      max_pts = std::max(max_pts, a.npts);
      max_nf = std::max(max_nf, s->nf);
    }
    pl.add(ops, [=](const FsiArgs* d, int c) { return launch_body_ops_multi<T>(d, c, max_pts, 0, st); });
    pl.add(mv, [=](const MatvecJob* d, int c) { return launch_matvec_multi(d, c, max_nf, st); });
  }
  if (!iter.empty()) {
    std::vector<FsiArgs> fa;
    std::vector<BeamJob> beams;
    std::vector<UpdateJob> upd;
    int max_pts = 0, max_m = 0, max_ub = 0;
    size_t beam_lds_max = 0;
    // The Schur assembly in classes of LDS size, one launch each: a launch's dynamic LDS is
    // its largest member's, and a workgroup sized for the largest system would hold a CU
    // alone for every member's rows
    constexpr int NSC = 4;
    const size_t sc_lim[NSC] = {20 * 1024, 40 * 1024, 80 * 1024, SCHUR_LDS_MAX};
    std::vector<FsiArgs> sc_fa[NSC];
    int sc_nf[NSC] = {0, 0, 0, 0};
    size_t sc_lds[NSC] = {0, 0, 0, 0};
    for (ib_solver* s : iter) {
      FsiArgs a = s->fa;
      a.gate = s->gate;
      fa.push_back(a);
      max_pts = std::max(max_pts, a.npts);
      const size_t l = schur_lds_bytes(a);
      if (l == 0) {
        b->last_error = "Schur assembly does not fit a workgroup";
        return IB_ERR_ARG;
      }
      int k = 0;
      while (l > sc_lim[k]) ++k;
      sc_fa[k].push_back(a);
      sc_nf[k] = std::max(sc_nf[k], s->nf);
      sc_lds[k] = std::max(sc_lds[k], l);
      for (size_t bi = 0; bi < s->bodies.size(); ++bi) {
        if (s->bodies[bi].kind != BODY_DEFORMABLE) continue;
        const int m = s->bodies[bi].m;
        beams.push_back(BeamJob{a, (int)bi, m});
        max_m = std::max(max_m, m);
        beam_lds_max = std::max(beam_lds_max, beam_lds(m));
      }
      const int nb = update_blocks(s->nf);
      upd.push_back(UpdateJob{a, s->cfg.newton_tol, s->cfg.newton_fixed_iter, nb});
      max_ub = std::max(max_ub, nb);
    }
    const size_t fa_off = pl.put(fa);
    size_t sc_off[NSC];
    for (int k = 0; k < NSC; ++k) sc_off[k] = sc_fa[k].empty() ? 0 : pl.put(sc_fa[k]);
    const size_t beam_off = beams.empty() ? 0 : pl.put(beams);
    const size_t upd_off = pl.put(upd);
    const int ni = (int)iter.size(), nbeam = (int)beams.size();
    for (int it = 0; it < K; ++it) {
      if (nbeam)
        pl.launches.push_back([=](const char* d) {
          return launch_ops_beam_multi<T>(reinterpret_cast<const FsiArgs*>(d + fa_off), ni,
                                          max_pts, reinterpret_cast<const BeamJob*>(d + beam_off),
                                          nbeam, max_m, beam_lds_max, it, st);
        });
      else
        pl.launches.push_back([=](const char* d) {
          return launch_body_ops_multi<T>(reinterpret_cast<const FsiArgs*>(d + fa_off), ni,
                                          max_pts, it, st);
        });
      for (int k = 0; k < NSC; ++k) {
        if (sc_fa[k].empty()) continue;
        const size_t off = sc_off[k], lds = sc_lds[k];
        const int cnt = (int)sc_fa[k].size(), mnf = sc_nf[k];
        pl.launches.push_back([=](const char* d) {
          return launch_schur_sd_multi(reinterpret_cast<const FsiArgs*>(d + off), cnt, mnf, lds,
                                       it, st);
        });
      }
      // Newton-Schulz refresh of the inverse into Xn, then the refinement (split by the
      // GEMM's k chunk and the refinement's LDS mode)
      std::vector<GemmJob> g1[2], g2[2];
      // refinements by LDS mode, and within a mode by the same LDS size classes as the
      // Schur assembly (a launch's LDS is its largest member's)
      std::vector<RefineJob> rj[3][NSC];
      int gmax_n[2] = {0, 0}, rnb[3][NSC] = {};
      size_t rlds[3][NSC] = {};
      for (ib_solver* s : iter) {
        const FsiArgs& a = s->fa;
        const int nf = s->nf;
        const bool refresh = refresh_at(s, it);
        const double* X = s->Minv;
        double* xcopy = nullptr;
        if (refresh) {
          const int k = nf <= GEMM_ONE_N ? 1 : 0;
          g1[k].push_back(GemmJob{a.M, s->Minv, s->W, nf, a.pm, 1, s->gate});
          g2[k].push_back(GemmJob{s->Minv, s->W, s->Xn, nf, a.pm, 0, s->gate});
          gmax_n[k] = std::max(gmax_n[k], nf);
          X = s->Xn;
          xcopy = s->Minv;
        }
        RefineShape sh;
        if (!refine_shape(nf, &sh)) {
          b->last_error = "Schur system too large for the refinement";
          return IB_ERR_ARG;
        }
        const int c = sh.two ? 2 : sh.cache ? 1 : 0;
        int k = 0;
        while (sh.lds > sc_lim[k]) ++k;
        rj[c][k].push_back(RefineJob{a.M, X, a.pm, s->rhs, s->f, nf, sh.rw, sh.tpr, REFINE_MAXIT,
                                     refine_guess(s, it), s->rinfo, s->rout, s->flags,
                                     s->gate, xcopy, sh.nb, s->barrier_arg()});
        rnb[c][k] = std::max(rnb[c][k], sh.nb);
        rlds[c][k] = std::max(rlds[c][k], sh.lds);
      }
      for (int k = 0; k < 2; ++k) {
        const int mn = gmax_n[k];
        pl.add(g1[k], [=](const GemmJob* d, int c) { return launch_gemm64_multi(d, c, mn, k, st); });
      }
      for (int k = 0; k < 2; ++k) {
        const int mn = gmax_n[k];
        pl.add(g2[k], [=](const GemmJob* d, int c) { return launch_gemm64_multi(d, c, mn, k, st); });
      }
      for (int c = 0; c < 3; ++c)
        for (int k = 0; k < NSC; ++k) {
          const int mb = rnb[c][k];
          const size_t l = rlds[c][k];
          pl.add(rj[c][k], [=](const RefineJob* d, int cnt) {
            return launch_refine_multi(d, cnt, mb, l, c, st);
          });
        }
      pl.launches.push_back([=](const char* d) {
        return launch_update_multi(reinterpret_cast<const UpdateJob*>(d + upd_off), ni, max_ub, it,
                                   K, st);
      });
    }
    pl.launches.push_back([=](const char* d) {
      return launch_finish_multi(reinterpret_cast<const FsiArgs*>(d + fa_off), ni, st);
    });
  }
  // The control blocks of the members iterating on the device are final after their FSI
  // iterations: gathered and copied to the host right there, so that the host reads them and
  // builds and queues the next step while the (gated) corrector and final transforms run.
  if (!iter.empty()) {
    std::vector<int*> ictl;
    for (ib_solver* s : iter) ictl.push_back(s->flags);
    ib_status rs0 = batch_reserve(b, 0, (int)ictl.size());
    if (rs0) return rs0;
    int* const dctl_target = b->dctl;
    int* const hctl_target = b->hctl;
    hipEvent_t const ready = b->ctl_ready;
    const size_t cb = ictl.size() * FsiCtl::BYTES;
    pl.add(ictl, [=](int* const* d, int c) { return launch_gather_ctl(d, c, dctl_target, st); });
    pl.launches.push_back([=](const char*) {
      const hipError_t e = hipMemcpyAsync(hctl_target, dctl_target, cb, hipMemcpyDeviceToHost, st);
      return e != hipSuccess ? e : hipEventRecord(ready, st);
    });
  }
  {
    // corrector source on level 0 (eqs. (20), (40)) for every member with bodies
    std::vector<SpreadJob<T>> sp;
    int gx = 0, gy = 0, mnf = 0;
    for (ib_solver* s : bodied) {
      mnf = std::max(mnf, s->nf);
      if (s->nf > SPREAD_ROWS_MAX) {
        b->last_error = "too many body rows for the spread";
        return IB_ERR_ARG;
      }
      FsiArgs a = s->fa;
      a.gate = gate_of(s);
      sp.push_back(SpreadJob<T>{a, s->blo, s->bhi, s->bilo, s->bihi, static_cast<T*>(s->work2),
                                s->pitch});
      gx = std::max(gx, (s->n - 1 + SPREAD_TILE_X - 1) / SPREAD_TILE_X);
      gy = std::max(gy, (s->bhi - s->blo + 1 + SPREAD_TILE_Y - 1) / SPREAD_TILE_Y);
    }
    pl.add(sp, [=](const SpreadJob<T>* d, int c) { return launch_spread_multi<T>(d, c, gx, gy, mnf, st); });
  }
  for (auto& q : groups) {
    std::vector<RowArgs<T>> rows;
    std::vector<ColArgs<T>> cols;
    std::vector<IdstJob<T>> fin;
    int maxrows = 0;
    for (ib_solver* s : q.m) {
      const int n = s->n, P = s->pitch, G = (int)s->lv.size();
      LevelState& L0 = s->lv[0];
      const int* gate = s->bodies.empty() ? nullptr : gate_of(s);
      if (!s->bodies.empty()) {
        RowArgs<T> r{};
        r.in = static_cast<T*>(s->work2);
        r.out = static_cast<T*>(s->work2);
        r.pi = r.po = P;
        r.r0 = s->blo;
        r.r1 = s->bhi;
        r.gate = gate;
        rows.push_back(r);
        maxrows = std::max(maxrows, s->bhi - s->blo + 1);
        ColArgs<T> c{};
        c.in = static_cast<T*>(s->work2);
        c.out = static_cast<T*>(s->work);
        c.pi = c.po = P;
        c.r0 = s->blo;
        c.r1 = s->bhi;
        c.alpha = (T)L0.alpha;
        c.scale = (T)(-s->cfg.dt * 4.0 / ((double)n * n));
        c.out2 = static_cast<T*>(s->workg);
        c.accumulate = 1;
        c.w0 = 1;
        c.w1 = n - 1;
        c.var = s->tune.col;
        c.gate = gate;
        cols.push_back(c);
      }
      RowArgs<T> r{};
      r.in = static_cast<T*>(s->work);
      r.pi = r.po = P;
      r.out = static_cast<T*>(L0.s);
      r.r0 = 1;
      r.r1 = n - 1;
      r.in2 = static_cast<T*>(s->workg);
      r.out2 = static_cast<T*>(L0.g);
      r.var = s->tune.idst;
      r.gate = gate;
      fin.push_back(IdstJob<T>{r, G > 1 ? static_cast<T*>(L0.sring) : nullptr, 1});
    }
    const int n = q.n, vc = q.vc, vi = q.vi;
    const void* tw = q.m[0]->tw;
    const void* lam = q.m[0]->lam;
    pl.add(rows, [=](const RowArgs<T>* d, int c) {
      return launch_rowdst_multi<T>(d, c, n, maxrows, tw, st);
    });
    pl.add(cols, [=](const ColArgs<T>* d, int c) {
      return launch_col_solve_multi<T>(d, c, n, vc, tw, lam, st);
    });
    pl.add(fin, [=](const IdstJob<T>* d, int c) {
      return launch_row_idst_multi<T>(d, c, n, n - 1, 1, vi, tw, st);
    });
  }
  ib_status rs0 = batch_reserve(b, pl.tab.size(), (int)iter.size());
  if (rs0) return rs0;

  // ---- tables to the device (one copy), then the launches
  const int k = b->slot;
  b->slot ^= 1;
  BCHK(hipEventSynchronize(b->copied[k]));  // the copy from this slot two steps ago is done
  std::memcpy(b->hbuf[k], pl.tab.data(), pl.tab.size());
  BCHK(hipMemcpyAsync(b->dbuf[k], b->hbuf[k], pl.tab.size(), hipMemcpyHostToDevice, st));
  BCHK(hipEventRecord(b->copied[k], st));
  for (auto& f : pl.launches) BCHK(f(b->dbuf[k]));
  b->launches += (int64_t)pl.launches.size();

  // ---- convergence of the members iterating on the device
  if (!iter.empty()) {
    // copied right after the FSI part (above); the corrector and final transforms may still run
    BCHK(hipEventSynchronize(b->ctl_ready));
    for (size_t i = 0; i < iter.size(); ++i) {
      ib_solver* s = iter[i];
      std::memcpy(s->hctl, reinterpret_cast<const char*>(b->hctl) + i * FsiCtl::BYTES,
                  FsiCtl::BYTES);
      int resume = -1;
      ib_status rs = fsi_after_ahead(s, &resume);
      if (!rs && resume >= 0) {
        // the launched iterations did not suffice: finish on the host as a lone step would
        s->fsi_resumes++;
        b->resumes++;
        rs = fsi_host<T>(s, resume);
        if (!rs) rs = final_transform_level0<T>(s);
      }
      if (rs) {
        s->failed = true;
        b->last_error = s->last_error;
        return rs;
      }
    }
  }
  for (ib_solver* s : stat) {
    s->iters_last = 1;
    s->delta_last = 0.0;
    s->iters_max = std::max(s->iters_max, 1);
  }
  for (ib_solver* s : ready) {
    const int G = (int)s->lv.size();
    for (int g = 0; g < G - 1; ++g) s->lv[g].gcur = 1 - s->lv[g].gcur;
    s->first = false;
    s->step++;
  }
  b->member_steps_batched += (int64_t)ready.size();
  return IB_OK;
}

#undef BCHK

}  // namespace

// ======================================================================== C ABI

// Measured choice of the single-precision transform kernel configurations for one grid
// size (process-wide, by n): every configuration of the right-hand side + row transform,
// the column solve and the inverse row transform runs on scratch buffers of a level's
// shape, and the fastest average launch time wins.  One solver measures at a time.
std::mutex g_tune_mu;
std::map<int, FlowTuning> g_tune;

ib_status tune_flow(ib_solver* s) {
  const int n = s->n, P = s->pitch;
  if (s->tune_forced) return IB_OK;
  s->tune = FlowTuning{};
  if (s->fp64 || s->ny != n || !ib::flow_variant_available(n, 0)) return IB_OK;
  std::lock_guard<std::mutex> lk(g_tune_mu);
  auto it = g_tune.find(n);
  if (it != g_tune.end()) {
    s->tune = it->second;
    return IB_OK;
  }
  const size_t full = (size_t)(n + 1) * P * 4, inner = (size_t)(n - 1) * P * 4;
  const size_t ring = (size_t)4 * (n + 1) * 4, edges = (size_t)4 * (n - 1) * 4;
  float* sf = static_cast<float*>(dalloc(s, full));
  float* gi = static_cast<float*>(dalloc(s, inner));
  float* hist = static_cast<float*>(dalloc(s, inner));
  float* out = static_cast<float*>(dalloc(s, inner));
  float* out2 = static_cast<float*>(dalloc(s, inner));
  float* gr = static_cast<float*>(dalloc(s, ring));
  float* gr2 = static_cast<float*>(dalloc(s, ring));
  float* lift = static_cast<float*>(dalloc(s, edges));
  hipEvent_t e0 = nullptr, e1 = nullptr;
  auto release = [&]() {
    for (void* p : {(void*)sf, (void*)gi, (void*)hist, (void*)out, (void*)out2, (void*)gr,
                    (void*)gr2, (void*)lift})
      dfree(s, p);
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
  };
  if (!sf || !gi || !hist || !out || !out2 || !gr || !gr2 || !lift) {
    release();
    return IB_ERR_OOM;
  }
  hipError_t e = hipSuccess;
  for (auto pr : {std::make_pair((void*)sf, full), std::make_pair((void*)gi, inner),
                  std::make_pair((void*)hist, inner), std::make_pair((void*)out, inner),
                  std::make_pair((void*)out2, inner), std::make_pair((void*)gr, ring),
                  std::make_pair((void*)gr2, ring), std::make_pair((void*)lift, edges)})
    if (e == hipSuccess) e = hipMemsetAsync(pr.first, 0, pr.second, s->stream);
  if (e == hipSuccess) e = hipEventCreate(&e0);
  if (e == hipSuccess) e = hipEventCreate(&e1);
  if (e != hipSuccess) {
    release();
    return hip_fail(s, e, "flow tuning set-up");
  }
  const double h = s->cfg.h;
  RhsArgs<float> a{};
  a.s = sf;
  a.g = gi;
  a.gring = gr;
  a.gring_new = gr2;
  a.hist_in = hist;
  a.hist_out = hist;
  a.out = out;
  a.n = n;
  a.ps = a.pg = a.pgf = a.ph = a.po = P;
  a.alpha = (float)(s->cfg.dt / (2.0 * s->cfg.re * h * h));
  a.dt = (float)s->cfg.dt;
  a.cn = (float)(-1.0 / (2.0 * h * h));
  ColArgs<float> c{};
  c.in = c.out = out;
  c.out2 = out2;
  c.lift = lift;
  c.pi = c.po = P;
  c.r0 = 1;
  c.r1 = n - 1;
  c.alpha = a.alpha;
  c.scale = (float)(4.0 / ((double)n * n));
  c.w0 = 1;
  c.w1 = n - 1;
  RowArgs<float> r{};
  r.in = out;
  r.in2 = out2;
  r.out = sf;
  r.out2 = gi;
  r.pi = r.po = P;
  r.r0 = 1;
  r.r1 = n - 1;
  constexpr int REPS = 3, K = 8;
  // average launch time of configuration v of kernel kind k (0 rhs, 1 col, 2 idst)
  auto measure = [&](int k, int v, double* us) -> hipError_t {
    auto launch = [&]() -> hipError_t {
      if (k == 0) {
        a.var = v;
        return launch_rhs_rowdst<float>(a, s->tw, s->stream);
      }
      if (k == 1) {
        c.var = v;
        return launch_col_solve<float>(c, n, 1, s->tw, s->lam, s->stream);
      }
      r.var = v;
      return launch_row_idst<float>(r, n, 1, s->tw, static_cast<float*>(gr), 1, s->stream);
    };
    double best = 1e30;
    for (int rep = 0; rep < REPS; ++rep) {
      hipError_t q = launch();  // warm-up
      if (q == hipSuccess) q = hipEventRecord(e0, s->stream);
      for (int i = 0; i < K && q == hipSuccess; ++i) q = launch();
      if (q == hipSuccess) q = hipEventRecord(e1, s->stream);
      if (q == hipSuccess) q = hipEventSynchronize(e1);
      float ms = 0.0f;
      if (q == hipSuccess) q = hipEventElapsedTime(&ms, e0, e1);
      if (q != hipSuccess) return q;
      best = std::min(best, 1e3 * ms / K);
    }
    *us = best;
    return hipSuccess;
  };
  FlowTuning t;
  t.n = n;
  double* tabs[3] = {t.rhs_us, t.col_us, t.idst_us};
  int* pick[3] = {&t.rhs, &t.col, &t.idst};
  for (int k = 0; k < 3 && e == hipSuccess; ++k) {
    if (k == 0 && s->gemm) continue;  // the matrix-core path has its own right-hand side pass
    const int kind = k == 1 ? 1 : 0;
    for (int v = 0; v < ib::FLOW_VARIANTS && e == hipSuccess; ++v)
      if (ib::flow_kind_variant_available(kind, v, n, 0)) e = measure(k, v, &tabs[k][v]);
    int b = 0;
    for (int v = 1; v < ib::FLOW_VARIANTS; ++v)
      if (tabs[k][v] > 0.0 && tabs[k][v] < tabs[k][b]) b = v;
    *pick[k] = b;
  }
  if (e == hipSuccess) e = hipStreamSynchronize(s->stream);
  release();
  if (e != hipSuccess) return hip_fail(s, e, "flow tuning");
  if (!s->gemm) g_tune[n] = t;
  s->tune = t;
  return IB_OK;
}

// No-slip residual of the last step and the force of every body, computed on the device
// (k_outputs) once per step and kept on the host, so that they stay readable after
// ib_release.  Nothing to do before the first step, without bodies, or once released.
template <typename T>
ib_status compute_outputs_t(ib_solver* s) {
  const size_t cnt = 1 + 2 * (size_t)s->fa.nbodies;
  if (!s->dout) {
    s->dout = static_cast<double*>(dalloc(s, cnt * 8));
    if (!s->dout) return IB_ERR_OOM;
  }
  HIPCHK(launch_outputs<T>(s->fa, static_cast<const T*>(s->lv[0].s), s->pitch, s->dout,
                           s->stream));
  s->h_out.assign(cnt, 0.0);
  HIPCHK(hipMemcpyAsync(s->h_out.data(), s->dout, cnt * 8, hipMemcpyDeviceToHost, s->stream));
  HIPCHK(hipStreamSynchronize(s->stream));
  s->out_step = s->step;
  return IB_OK;
}

ib_status compute_outputs(ib_solver* s) {
  if (!s->prepared || s->released || !s->allocated || s->bodies.empty() || s->step == 0 ||
      s->failed || s->out_step == s->step)
    return IB_OK;
  return s->fp64 ? compute_outputs_t<double>(s) : compute_outputs_t<float>(s);
}

extern "C" {

const char* ib_status_str(ib_status st) {
  switch (st) {
    case IB_OK: return "ok";
    case IB_ERR_ARG: return "invalid argument";
    case IB_ERR_STATE: return "invalid call order or failed solver";
    case IB_ERR_OOM: return "out of device memory";
    case IB_ERR_HIP: return "HIP runtime error";
    case IB_ERR_NOT_CONVERGED: return "FSI iteration did not converge";
    case IB_ERR_OUT_OF_SUBDOMAIN: return "body left the sub-domain";
    case IB_ERR_NEAR_BOUNDARY: return "delta support reaches the finest level's boundary";
    case IB_ERR_NONFINITE: return "non-finite value";
    case IB_ERR_CAPACITY: return "output buffer too small";
    case IB_ERR_BUDGET: return "over the device-memory budget";
    case IB_ERR_SCRATCH: return "larger than the fixed device scratch of an allocation-free call";
    default: return "unknown status";
  }
}

ib_status ib_create(const ib_config* cfg, const ib_allocator* alloc, void* hip_stream,
                    ib_solver** out) {
  if (!cfg || !out) return IB_ERR_ARG;
  *out = nullptr;
  const int cny = cfg->ny > 0 ? cfg->ny : cfg->n;
  if (cfg->ny < 0 || !supported_n(cny) || cny % 4 != 0 ||
      (cny != cfg->n && cfg->precision == IB_FP32_FLOW_BF16_DST))
    return IB_ERR_ARG;
  // double precision up to 2000 cells per axis; the matrix-core transforms up to 1280
  if (cfg->precision == IB_FP64 && (!supported_n_fp64(cfg->n) || !supported_n_fp64(cny)))
    return IB_ERR_ARG;
  if (cfg->precision == IB_FP32_FLOW_BF16_DST && cfg->n > 1280) return IB_ERR_ARG;
  if (!supported_n(cfg->n) || cfg->n % 4 != 0 || cfg->levels < 1 || cfg->levels > 12 ||
      !(cfg->h > 0) || !(cfg->dt > 0) || !(cfg->re > 0) ||
      (cfg->precision != IB_FP64 && cfg->precision != IB_FP32_FLOW &&
       cfg->precision != IB_FP32_FLOW_BF16_DST) || cfg->schur_mode < 0 ||
      cfg->schur_mode > 2 || (cfg->delta != IB_DELTA_ROMA3 && cfg->delta != IB_DELTA_PESKIN4))
    return IB_ERR_ARG;
  ib_solver* s = new ib_solver();
  s->cfg = *cfg;
  if (s->cfg.newton_tol <= 0) s->cfg.newton_tol = 1e-7;
  if (s->cfg.newton_max_iter <= 0) s->cfg.newton_max_iter = 20;
  if (s->cfg.drop_tol < 0) s->cfg.drop_tol = 0.007;
  if (alloc && alloc->alloc && alloc->free) {
    s->alloc = *alloc;
    s->has_alloc = true;
  }
  s->stream = static_cast<hipStream_t>(hip_stream);
  s->n = cfg->n;
  s->ny = cny;
  s->fp64 = cfg->precision == IB_FP64;
  s->gemm = cfg->precision == IB_FP32_FLOW_BF16_DST;
  s->es = s->fp64 ? 8 : 4;
  s->pitch = round_up(s->n + 1, 64);
  for (int g = 0; g < cfg->levels; ++g) {
    LevelState L;
    L.h = cfg->h * std::ldexp(1.0, g);
    L.alpha = cfg->dt / (2.0 * cfg->re * L.h * L.h);
    s->lv.push_back(L);
  }
  *out = s;
  return IB_OK;
}

ib_status ib_add_rigid(ib_solver* s, int32_t m, const double* xy, double ds, const double* u_b,
                       int32_t* body_id) {
  if (check(s) || m < 1 || !xy || !(ds > 0)) return IB_ERR_ARG;
  if (s->prepared) return IB_ERR_STATE;
  HostBody b;
  b.kind = BODY_RIGID;
  b.m = m;
  b.ds = ds;
  b.xy.assign(xy, xy + 2 * m);
  if (u_b) b.ub.assign(u_b, u_b + 2 * m);
  s->bodies.push_back(b);
  if (body_id) *body_id = (int32_t)s->bodies.size() - 1;
  return IB_OK;
}

ib_status ib_add_moving_rigid(ib_solver* s, int32_t m, const double* xy_ref, double ds,
                              ib_motion_fn motion, void* ctx, int32_t* body_id) {
  if (check(s) || m < 1 || !xy_ref || !(ds > 0) || !motion) return IB_ERR_ARG;
  if (s->prepared) return IB_ERR_STATE;
  HostBody b;
  b.kind = BODY_MOVING;
  b.m = m;
  b.ds = ds;
  b.xy.assign(xy_ref, xy_ref + 2 * m);
  b.motion = motion;
  b.motion_ctx = ctx;
  s->bodies.push_back(b);
  if (body_id) *body_id = (int32_t)s->bodies.size() - 1;
  return IB_OK;
}

ib_status ib_add_torsional(ib_solver* s, int32_t m, double hinge_x, double hinge_y, double length,
                           double theta0, double inertia, double stiffness, double damping,
                           double theta, double phi, int32_t* body_id) {
  if (check(s) || m < 2 || !(length > 0) || !(inertia > 0)) return IB_ERR_ARG;
  if (s->prepared) return IB_ERR_STATE;
  HostBody b;
  b.kind = BODY_TORSIONAL;
  b.m = m;
  b.ds = length / (m - 1);
  b.hx = hinge_x;
  b.hy = hinge_y;
  b.length = length;
  b.theta0 = theta0;
  b.inertia = inertia;
  b.stiffness = stiffness;
  b.damping = damping;
  b.theta = theta;
  b.phi = phi;
  s->bodies.push_back(b);
  if (body_id) *body_id = (int32_t)s->bodies.size() - 1;
  return IB_OK;
}

ib_status ib_add_mounted_torsional(ib_solver* s, int32_t m, int32_t driver, double hinge_bx,
                                  double hinge_by, double theta_rel, double length,
                                  double inertia, double stiffness, double damping, double mass,
                                  double cg, double theta, double phi, int32_t* body_id) {
  if (check(s) || m < 2 || !(length > 0) || !(inertia > 0) || !(mass >= 0) || driver < 0 ||
      driver >= (int32_t)s->bodies.size() || s->bodies[driver].kind != BODY_MOVING ||
      !std::isfinite(hinge_bx) || !std::isfinite(hinge_by) || !std::isfinite(theta_rel) ||
      !std::isfinite(cg))
    return IB_ERR_ARG;
  if (s->prepared) return IB_ERR_STATE;
  HostBody b;
  b.kind = BODY_TORSIONAL;
  b.m = m;
  b.ds = length / (m - 1);
  b.length = length;
  b.inertia = inertia;
  b.stiffness = stiffness;
  b.damping = damping;
  b.mass = mass;
  b.cg = cg;
  b.theta = theta;
  b.phi = phi;
  b.driver = driver;
  b.hbx = hinge_bx;
  b.hby = hinge_by;
  b.theta_rel = theta_rel;
  s->bodies.push_back(b);
  if (body_id) *body_id = (int32_t)s->bodies.size() - 1;
  return IB_OK;
}

ib_status ib_add_deformable(ib_solver* s, int32_t m, const double* xy_ref, double mass, double ei,
                            double ea, const double* xy0, const double* rot0, int32_t* body_id) {
  if (check(s) || m < 2 || m > 201 || !xy_ref || !xy0 || !rot0 || !(mass > 0) || !(ei > 0) ||
      !(ea > 0))
    return IB_ERR_ARG;
  if (s->prepared) return IB_ERR_STATE;
  HostBody b;
  b.kind = BODY_DEFORMABLE;
  b.m = m;
  b.xy_ref.assign(xy_ref, xy_ref + 2 * m);
  b.xy0.assign(xy0, xy0 + 2 * m);
  b.rot0.assign(rot0, rot0 + m);
  double len = 0;
  for (int k = 0; k + 1 < m; ++k)
    len += std::hypot(xy_ref[2 * k + 2] - xy_ref[2 * k], xy_ref[2 * k + 3] - xy_ref[2 * k + 1]);
  b.ds = len / (m - 1);
  b.mass = mass;
  b.ei = ei;
  b.ea = ea;
  s->bodies.push_back(b);
  if (body_id) *body_id = (int32_t)s->bodies.size() - 1;
  return IB_OK;
}

ib_status ib_set_subdomain(ib_solver* s, double x0, double x1, double y0, double y1) {
  if (check(s) || !(x1 > x0) || !(y1 > y0)) return IB_ERR_ARG;
  if (s->prepared) return IB_ERR_STATE;
  if ((int)s->sd_rects.size() >= ib::SD_MAX_BOXES) {
    s->last_error = "more than 8 sub-domain rectangles";
    return IB_ERR_ARG;
  }
  s->has_sd = true;
  s->sd_rects.push_back({x0, x1, y0, y1});
  return IB_OK;
}

ib_status ib_set_vorticity(ib_solver* s, int32_t level, const double* omega) {
  if (check(s) || level < 0 || level >= (int)s->lv.size() || !omega) return IB_ERR_ARG;
  if (s->prepared) return IB_ERR_STATE;
  if ((int)s->omega0.size() <= level) s->omega0.resize(level + 1);
  s->omega0[level].assign(omega, omega + (size_t)(s->n - 1) * (s->ny - 1));
  return IB_OK;
}

ib_status ib_prepare(ib_solver* s) {
  HipShared hip_lock;
  if (check(s)) return IB_ERR_ARG;
  if (s->prepared || s->released) return IB_ERR_STATE;
  if (s->ny != s->n && !s->bodies.empty()) {
    s->last_error = "bodies need square levels (ny = n)";
    return IB_ERR_ARG;
  }
  if (s->n > 1280 && !s->bodies.empty()) {
    // the offline operators are built in double precision with the square kernels of n
    s->last_error = "bodies need at most 1280 cells per side";
    return IB_ERR_ARG;
  }
  ib_status st = s->allocated ? IB_OK : alloc_state(s);
  if (st == IB_OK) st = tune_flow(s);
  if (st == IB_OK) st = s->fp64 ? do_prepare<double>(s) : do_prepare<float>(s);
  if (st) {
    s->failed = true;
    return st;
  }
  s->prepared = true;
  return IB_OK;
}

ib_status ib_step(ib_solver* s, int32_t nsteps) {
  if (check(s) || nsteps < 0) return IB_ERR_ARG;
  if (!s->prepared || s->failed || s->released) return IB_ERR_STATE;
  struct Stepping {
    Stepping() { g_stepping.fetch_add(1, std::memory_order_relaxed); }
    ~Stepping() { g_stepping.fetch_sub(1, std::memory_order_relaxed); }
  } stepping;
  for (int k = 0; k < nsteps; ++k) {
    const StepPlan p = plan_step(s);
    ib_status st = IB_OK;
    if (needs_record(s, p)) {
      // only when no other thread is inside the library's HIP calls: recording never
      // waits (under load from other solvers the step simply runs without a graph)
      std::unique_lock<std::shared_mutex> lk(g_hip_mu, std::try_to_lock);
      if (lk.owns_lock()) st = s->fp64 ? record_step<double>(s, p) : record_step<float>(s, p);
    }
    if (!st) {
      HipShared lk;
      const bool more = k + 1 < nsteps;
      st = s->fp64 ? do_step<double>(s, p, more) : do_step<float>(s, p, more);
    }
    if (st) {
      s->failed = true;
      if (s->side_ahead) {
        // levels launched for a step that will not run: let them finish
        (void)hipStreamSynchronize(s->side);
        s->side_ahead = false;
      }
      return st;
    }
  }
  return IB_OK;
}

ib_status ib_sync(ib_solver* s) {
  HipShared hip_lock;
  if (check(s)) return IB_ERR_ARG;
  hipError_t e = hipStreamSynchronize(s->stream);
  return e == hipSuccess ? IB_OK : hip_fail(s, e, "hipStreamSynchronize");
}

ib_status ib_read_stresses(ib_solver* s, int32_t body_id, double* f, int64_t cap) {
  HipShared hip_lock;
  if (check(s) || !f || body_id < 0 || body_id >= (int)s->bodies.size()) return IB_ERR_ARG;
  if (!s->prepared || (!s->f && !s->released)) return IB_ERR_STATE;
  int pt0 = 0;
  for (int k = 0; k < body_id; ++k) pt0 += s->bodies[k].m;
  const int m = s->bodies[body_id].m;
  if (cap < 2 * m) return IB_ERR_CAPACITY;
  if (s->released) {
    std::memcpy(f, s->h_f.data() + 2 * pt0, (size_t)2 * m * 8);
    return IB_OK;
  }
  HIPCHK(hipStreamSynchronize(s->stream));
  HIPCHK(hipMemcpy(f, s->f + 2 * pt0, (size_t)2 * m * 8, hipMemcpyDeviceToHost));
  return IB_OK;
}

ib_status ib_read_force(ib_solver* s, int32_t body_id, double* out, int64_t cap) {
  HipShared hip_lock;
  if (check(s) || !out || body_id < 0 || body_id >= (int)s->bodies.size()) return IB_ERR_ARG;
  if (!s->prepared) return IB_ERR_STATE;
  if (cap < 2) return IB_ERR_CAPACITY;
  const ib_status st = compute_outputs(s);
  if (st) return st;
  if (s->out_step < 0 || s->h_out.size() < 3 + 2 * (size_t)body_id) {
    out[0] = out[1] = 0.0;  // no step taken yet
    return IB_OK;
  }
  out[0] = s->h_out[1 + 2 * body_id];
  out[1] = s->h_out[2 + 2 * body_id];
  return IB_OK;
}

ib_status ib_read_deflection(ib_solver* s, int32_t body_id, double* out, int64_t cap) {
  HipShared hip_lock;
  if (check(s) || !out || body_id < 0 || body_id >= (int)s->bodies.size()) return IB_ERR_ARG;
  if (!s->prepared) return IB_ERR_STATE;
  if (!s->released) HIPCHK(hipStreamSynchronize(s->stream));
  const HostBody& hb = s->bodies[body_id];
  int tors = 0, dof = 0;
  for (int k = 0; k < body_id; ++k) {
    if (s->bodies[k].kind == BODY_TORSIONAL) ++tors;
    if (s->bodies[k].kind == BODY_DEFORMABLE) dof += 3 * s->bodies[k].m;
  }
  if (hb.kind == BODY_TORSIONAL) {
    if (cap < 3) return IB_ERR_CAPACITY;
    if (s->released) std::memcpy(out, s->h_tors.data() + tors * TS_COUNT, 3 * 8);
    else HIPCHK(hipMemcpy(out, s->fa.tors + tors * TS_COUNT, 3 * 8, hipMemcpyDeviceToHost));
  } else if (hb.kind == BODY_DEFORMABLE) {
    if (cap < 3 * hb.m) return IB_ERR_CAPACITY;
    if (s->released) std::memcpy(out, s->h_chi.data() + dof, (size_t)3 * hb.m * 8);
    else HIPCHK(hipMemcpy(out, s->fa.chi + dof, (size_t)3 * hb.m * 8, hipMemcpyDeviceToHost));
  } else if (hb.kind == BODY_MOVING) {
    // point positions at the pose of the last step's time level
    if (cap < 2 * hb.m) return IB_ERR_CAPACITY;
    const double c = std::cos(hb.pose[2]), sn = std::sin(hb.pose[2]);
    for (int k = 0; k < hb.m; ++k) {
      const double rx = hb.xy[2 * k], ry = hb.xy[2 * k + 1];
      out[2 * k] = hb.pose[0] + c * rx - sn * ry;
      out[2 * k + 1] = hb.pose[1] + sn * rx + c * ry;
    }
  } else {
    if (cap < 2 * hb.m) return IB_ERR_CAPACITY;
    std::memcpy(out, hb.xy.data(), (size_t)2 * hb.m * 8);
  }
  return IB_OK;
}

ib_status ib_read_streamfunction(ib_solver* s, int32_t level, double* out, int64_t cap) {
  HipShared hip_lock;
  if (check(s) || !out || level < 0 || level >= (int)s->lv.size()) return IB_ERR_ARG;
  if (!s->allocated) return IB_ERR_STATE;
  const int n = s->n, ny = s->ny;
  if (cap < (int64_t)(n + 1) * (ny + 1)) return IB_ERR_CAPACITY;
  HIPCHK(hipStreamSynchronize(s->stream));
  std::vector<char> buf((size_t)(ny + 1) * s->pitch * s->es);
  HIPCHK(hipMemcpy(buf.data(), s->lv[level].s, buf.size(), hipMemcpyDeviceToHost));
  for (int j = 0; j <= ny; ++j)
    for (int i = 0; i <= n; ++i) {
      const size_t k = (size_t)j * s->pitch + i;
      out[(size_t)j * (n + 1) + i] =
          s->fp64 ? reinterpret_cast<double*>(buf.data())[k] : reinterpret_cast<float*>(buf.data())[k];
    }
  return IB_OK;
}

ib_status read_vorticity_impl(ib_solver* s, int32_t level, double* out, int64_t cap) {
  if (check(s) || !out || level < 0 || level >= (int)s->lv.size()) return IB_ERR_ARG;
  const int n = s->n, ny = s->ny;
  if (cap < (int64_t)(n - 1) * (ny - 1)) return IB_ERR_CAPACITY;
  if (s->released) {
    if (level != 0) return IB_ERR_STATE;
    std::memcpy(out, s->h_vort0.data(), s->h_vort0.size() * 8);
    return IB_OK;
  }
  if (!s->allocated) return IB_ERR_STATE;
  HIPCHK(hipStreamSynchronize(s->stream));
  std::vector<char> buf((size_t)(ny - 1) * s->pitch * s->es);
  HIPCHK(hipMemcpy(buf.data(), s->lv[level].g, buf.size(), hipMemcpyDeviceToHost));
  const double h = s->lv[level].h;
  const double inv = 1.0 / (h * h);
  for (int j = 0; j < ny - 1; ++j)
    for (int i = 0; i < n - 1; ++i) {
      const size_t k = (size_t)j * s->pitch + i;
      const double g = s->fp64 ? reinterpret_cast<double*>(buf.data())[k]
                               : reinterpret_cast<float*>(buf.data())[k];
      out[(size_t)j * (n - 1) + i] = g * inv;
    }
  return IB_OK;
}

ib_status ib_read_vorticity(ib_solver* s, int32_t level, double* out, int64_t cap) {
  HipShared hip_lock;
  return read_vorticity_impl(s, level, out, cap);
}

ib_status ib_batch_create(ib_solver* const* members, int32_t count, void* hip_stream,
                          ib_batch** out) {
  HipShared hip_lock;
  if (!out || !members || count < 1) return IB_ERR_ARG;
  *out = nullptr;
  for (int i = 0; i < count; ++i) {
    ib_solver* s = members[i];
    if (!s) return IB_ERR_ARG;
    for (int j = 0; j < i; ++j)
      if (members[j] == s) return IB_ERR_ARG;
    // square levels of the batched kernels' sizes only
    if (s->fp64 != members[0]->fp64 || s->ny != s->n || s->n > 1280) return IB_ERR_ARG;
    if (!s->prepared || s->failed || s->released) return IB_ERR_STATE;
  }
  hipStream_t st = static_cast<hipStream_t>(hip_stream);
  for (int i = 0; i < count; ++i) {
    ib_solver* s = members[i];
    if (s->stream != st) {
      hipError_t e = hipStreamSynchronize(s->stream);  // work queued on the old stream
      if (e != hipSuccess) return hip_fail(s, e, "hipStreamSynchronize");
      s->stream = st;
    }
  }
  ib_batch* b = new ib_batch();
  b->mem.assign(members, members + count);
  b->stream = st;
  b->fp64 = members[0]->fp64;
  for (auto& e : b->copied)
    if (hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess) {
      for (auto f : b->copied)
        if (f) (void)hipEventDestroy(f);
      delete b;
      return IB_ERR_HIP;
    }
  if (hipEventCreateWithFlags(&b->ctl_ready, hipEventDisableTiming) != hipSuccess) {
    for (auto f : b->copied) (void)hipEventDestroy(f);
    delete b;
    return IB_ERR_HIP;
  }
  *out = b;
  return IB_OK;
}

ib_status ib_batch_step(ib_batch* b, int32_t nsteps) {
  if (!b || nsteps < 0) return IB_ERR_ARG;
  HipShared hip_lock;
  for (ib_solver* s : b->mem)
    if (!s->prepared || s->failed || s->released) {
      b->last_error = "a member is not prepared, has failed or was released";
      return IB_ERR_STATE;
    }
  for (int k = 0; k < nsteps; ++k) {
    ib_status st = b->fp64 ? batch_step<double>(b) : batch_step<float>(b);
    if (st) return st;
    b->steps++;
  }
  return IB_OK;
}

ib_status ib_batch_get_stats(const ib_batch* b, ib_batch_stats* out) {
  if (!b || !out) return IB_ERR_ARG;
  out->steps = b->steps;
  out->member_steps_batched = b->member_steps_batched;
  out->member_steps_alone = b->member_steps_alone;
  out->launches = b->launches;
  out->fsi_resumes = b->resumes;
  return IB_OK;
}

const char* ib_batch_last_error(const ib_batch* b) {
  if (!b) return "null batch";
  return b->last_error.c_str();
}

ib_status ib_batch_destroy(ib_batch* b) {
  if (!b) return IB_ERR_ARG;
  HipShared hip_lock;
  (void)hipStreamSynchronize(b->stream);
  batch_free_buffers(b);
  if (b->dctl) (void)hipFree(b->dctl);
  if (b->hctl) (void)hipHostFree(b->hctl);
  for (auto e : b->copied)
    if (e) (void)hipEventDestroy(e);
  if (b->ctl_ready) (void)hipEventDestroy(b->ctl_ready);
  delete b;
  return IB_OK;
}

const char* ib_last_error(const ib_solver* s) {
  if (!s) return "null solver";
  return s->last_error.c_str();
}

ib_status ib_get_stats(ib_solver* s, ib_stats* out) {
  if (check(s) || !out) return IB_ERR_ARG;
  {
    HipShared hip_lock;
    const ib_status st = compute_outputs(s);
    if (st) return st;
  }
  std::memset(out, 0, sizeof(*out));
  out->converged = s->bodies.empty() || s->step == 0 || s->delta_last <= s->cfg.newton_tol;
  if (s->out_step >= 0 && !s->h_out.empty()) {
    out->noslip_resid = s->h_out[0];
    const size_t nb = (s->h_out.size() - 1) / 2;
    for (size_t b = 0; b < nb; ++b) {
      out->force[0] += s->h_out[1 + 2 * b];
      out->force[1] += s->h_out[2 + 2 * b];
    }
  }
  out->step = s->step;
  out->newton_iters = s->iters_last;
  out->newton_iters_max = s->iters_max;
  out->newton_delta = s->delta_last;
  out->subdomain_points = s->use_sd ? 2 * (int64_t)s->sd_total : 0;
  out->subdomain_nnz = s->bp_nnz;
  out->prepare_seconds = s->prepare_seconds;
  out->refine_iters = s->hrinfo ? (int32_t)s->hrinfo[1] : 0;
  out->refine_residual = s->hrinfo ? s->hrinfo[0] : 0.0;
  out->inverse_rebuilds = s->inverse_rebuilds;
  out->operator_source = s->op ? s->op_source : -1;
  out->graph_launches = s->graph_launches;
  out->graph_captures = s->graph_captures;
  out->fsi_resumes = s->fsi_resumes;
  out->solve_fallbacks = s->solve_fallbacks;
  out->solve_by_lu = s->lu_always ? 1 : 0;
  return IB_OK;
}

ib_status ib_set_option(ib_solver* s, int32_t option, int64_t value) {
  HipShared hip_lock;
  if (option == IB_OPT_BARRIER_SPIN) {
    if (check(s) || value < 0 || value > (int64_t(1) << 40)) return IB_ERR_ARG;
    s->barrier_spin = (long)value;
    destroy_graphs(s);
    return IB_OK;
  }
  if (option == IB_OPT_BARRIER_FORCE_TIMEOUT) {
    if (check(s) || value < 0 || value > 1) return IB_ERR_ARG;
    s->barrier_force = value != 0;
    destroy_graphs(s);
    return IB_OK;
  }
  const int vmax = option == IB_OPT_REFRESH_EVERY_ITER || option == IB_OPT_TOP_AHEAD ? 2 : 1;
  if (check(s) || value < 0 || value > vmax) return IB_ERR_ARG;
  if (option == IB_OPT_FSI_AHEAD) {
    s->fsi_ahead = value != 0;
    destroy_graphs(s);
    return IB_OK;
  }
  if (option == IB_OPT_GRAPHS) {
    s->graphs = value != 0;
    destroy_graphs(s);
    return IB_OK;
  }
  if (option == IB_OPT_REFRESH_EVERY_ITER) {
    s->refresh_mode = (int)value;
    destroy_graphs(s);
    return IB_OK;
  }
  if (option == IB_OPT_TOP_AHEAD) {
    s->ahead_mode = (int)value;
    return IB_OK;
  }
  return IB_ERR_ARG;
}

ib_status ib_get_flow_tuning(ib_solver* s, ib_flow_tuning* out) {
  if (check(s) || !out) return IB_ERR_ARG;
  std::memset(out, 0, sizeof(*out));
  static_assert(IB_FLOW_VARIANTS == ib::FLOW_VARIANTS, "variant count");
  out->n = s->tune.n;
  out->rhs_variant = s->tune.rhs;
  out->col_variant = s->tune.col;
  out->idst_variant = s->tune.idst;
  for (int v = 0; v < IB_FLOW_VARIANTS; ++v) {
    out->rhs_us[v] = s->tune.rhs_us[v];
    out->col_us[v] = s->tune.col_us[v];
    out->idst_us[v] = s->tune.idst_us[v];
  }
  return IB_OK;
}

ib_status ib_set_flow_variants(ib_solver* s, int32_t rhs, int32_t col, int32_t idst) {
  HipShared hip_lock;
  if (check(s)) return IB_ERR_ARG;
  const int32_t v[3] = {rhs, col, idst};
  for (int k = 0; k < 3; ++k) {
    if (v[k] < -1 || v[k] >= IB_FLOW_VARIANTS) return IB_ERR_ARG;
    if (v[k] > 0 && (s->ny != s->n ||
                     !ib::flow_kind_variant_available(k == 1 ? 1 : 0, v[k], s->n, s->fp64 ? 1 : 0)))
      return IB_ERR_ARG;
  }
  if (rhs > 0 && s->gemm) return IB_ERR_ARG;
  if (rhs >= 0) s->tune.rhs = rhs;
  if (col >= 0) s->tune.col = col;
  if (idst >= 0) s->tune.idst = idst;
  s->tune_forced = true;
  destroy_graphs(s);  // recorded steps launch the previous configurations
  return IB_OK;
}

ib_status ib_flow_variant_info(int32_t kind, int32_t variant, int32_t* width, int32_t* threads,
                               int32_t* max_radix) {
  if ((kind != 0 && kind != 1) || variant < 0 ||
      variant >= (kind == 0 ? ib::ROW_VARIANT_COUNT : ib::COL_VARIANT_COUNT) || !width ||
      !threads || !max_radix)
    return IB_ERR_ARG;
  const ib::FlowVariant& f = kind == 0 ? ib::ROW_VARIANTS[variant] : ib::COL_VARIANTS[variant];
  *width = f.width;
  *threads = f.nt;
  *max_radix = f.maxr;
  return IB_OK;
}

ib_status ib_set_kernel_timing(ib_solver* s, int32_t enable) {
  HipShared hip_lock;
  if (check(s)) return IB_ERR_ARG;
  harvest_events(s);
  s->timing = enable != 0;
  for (int k = 0; k < IB_K_CLASSES; ++k) {
    s->t_count[k] = 0;
    s->t_ms[k] = 0.0;
  }
  return IB_OK;
}

ib_status ib_get_kernel_timing(ib_solver* s, int32_t kernel_class, int64_t* launches,
                               double* total_ms) {
  HipShared hip_lock;
  if (check(s) || kernel_class < 0 || kernel_class >= IB_K_CLASSES || !launches || !total_ms)
    return IB_ERR_ARG;
  harvest_events(s);
  *launches = s->t_count[kernel_class];
  *total_ms = s->t_ms[kernel_class];
  return IB_OK;
}

ib_status ib_set_stream(ib_solver* s, void* hip_stream) {
  HipShared hip_lock;
  if (check(s)) return IB_ERR_ARG;
  if (s->allocated) HIPCHK(hipStreamSynchronize(s->stream));  // work queued on the old stream
  s->stream = static_cast<hipStream_t>(hip_stream);
  return IB_OK;
}

ib_status ib_release(ib_solver* s) {
  HipShared hip_lock;
  if (check(s)) return IB_ERR_ARG;
  if (s->released) return IB_OK;
  if (s->allocated) {
    HIPCHK(hipStreamSynchronize(s->stream));
    if (s->side) HIPCHK(hipStreamSynchronize(s->side));
    destroy_graphs(s);
    {
      const ib_status st = compute_outputs(s);
      if (st) return st;
    }
    if (s->prepared && s->f) {
      s->h_f.resize(s->nf);
      HIPCHK(hipMemcpy(s->h_f.data(), s->f, (size_t)s->nf * 8, hipMemcpyDeviceToHost));
      s->h_tors.resize((size_t)s->ntors * TS_COUNT);
      if (s->ntors)
        HIPCHK(hipMemcpy(s->h_tors.data(), s->fa.tors, s->h_tors.size() * 8, hipMemcpyDeviceToHost));
      s->h_chi.resize(s->ndof);
      if (s->ndof)
        HIPCHK(hipMemcpy(s->h_chi.data(), s->fa.chi, s->h_chi.size() * 8, hipMemcpyDeviceToHost));
    }
    std::vector<double> v((size_t)(s->n - 1) * (s->ny - 1));
    ib_status st = read_vorticity_impl(s, 0, v.data(), (int64_t)v.size());
    if (st) return st;
    s->h_vort0.swap(v);
  }
  harvest_events(s);
  while (!s->allocs.empty()) dfree(s, s->allocs.back().first);
  s->f = nullptr;
  s->dout = nullptr;
  s->allocated = false;
  s->released = true;
  return IB_OK;
}

ib_status ib_estimate_bytes(const ib_solver* s, int64_t* resident, int64_t* peak) {
  if (!s || !resident || !peak) return IB_ERR_ARG;
  const int n = s->n, ny = s->ny, G = (int)s->lv.size();
  const size_t es = s->es, P = s->pitch;
  const size_t full = (size_t)(ny + 1) * P * es, inner = (size_t)(ny - 1) * P * es;
  const size_t ring = (size_t)ring_len(n, ny) * es, lift = (size_t)(2 * (n - 1) + 2 * (ny - 1)) * es;
  size_t r = (size_t)G * (full + 2 * inner + 3 * ring);
  r += 3 * inner + full + lift + 2 * (size_t)2 * n * (8 + es);
  if (ny != n) r += (size_t)2 * ny * (8 + es) + (size_t)(n + 1) * es;  // the y tables
  // scratch of the levels launched ahead (three or more levels)
  if (G >= 3 && !s->gemm) r += 2 * inner + lift;
  if (s->gemm) {
    // split sine matrix (two BF16 copies of kpad^2) and two FP32 product buffers
    const size_t kp = (size_t)(n - 1 + 63) / 64 * 64;
    r += 2 * kp * kp * 2 + 2 * (size_t)(n - 1) * P * 4 + (size_t)(n + 1) * 4;
  }
  size_t npts = 0, ndef_y = 0, app = 0;
  for (auto& hb : s->bodies) {
    npts += hb.m;
    if (hb.kind == BODY_DEFORMABLE) ndef_y += (size_t)(3 * hb.m) * (2 * hb.m + 1);
    if (hb.kind == BODY_RIGID) app += hb.m;
  }
  const size_t nf = 2 * npts, pm = (nf + 7) / 8 * 8;
  size_t peak_extra = 0;
  if (nf) {
    r += 5 * nf * pm * 8 + nf * (16 * 8 + 3 * 4 + 4 * 12 + 4 * 8) + ndef_y * 8 + (1 << 20);
    if (s->has_sd) {
      // B' rows and an allowance of 800 stored entries per row (about 750 measured at
      // the drop tolerance 0.007), plus the offline batch buffers
      const double h = s->cfg.h;
      size_t grid = 0;
      for (const auto& r : s->sd_rects)
        grid += ((size_t)((r[1] - r[0]) / h) + 3) * ((size_t)((r[3] - r[2]) / h) + 3);
      const size_t rows = 2 * (grid + app);
      const double scale = s->cfg.drop_tol > 0 ? std::min(4.0, 0.007 / s->cfg.drop_tol) : 4.0;
      r += rows * (size_t)(800 * scale) * 12 + rows * 12;
      peak_extra = (size_t)1 << 30;
    } else {
      peak_extra = std::min<size_t>((size_t)1 << 30, nf * ((size_t)(2 * n + 6) * P * 8 + nf * 8));
    }
  }
  *resident = (int64_t)r;
  *peak = (int64_t)(r + peak_extra);
  return IB_OK;
}

// Serialised operator: "IBOP0001", then int64 counts (key, ptr, col, val) and the arrays.
ib_status ib_export_operator(ib_solver* s, void* buf, int64_t cap, int64_t* used) {
  if (check(s) || !used) return IB_ERR_ARG;
  if (!s->op) return IB_ERR_STATE;
  const OpData& d = *s->op;
  const int64_t size = 8 + 4 * 8 + (int64_t)(d.key.size() * 8 + d.ptr.size() * 8 +
                                             d.col.size() * 4 + d.val.size() * 8);
  *used = size;
  if (!buf || cap < size) return IB_ERR_CAPACITY;
  char* p = static_cast<char*>(buf);
  std::memcpy(p, "IBOP0001", 8);
  p += 8;
  const int64_t cnt[4] = {(int64_t)d.key.size(), (int64_t)d.ptr.size(), (int64_t)d.col.size(),
                          (int64_t)d.val.size()};
  std::memcpy(p, cnt, sizeof(cnt));
  p += sizeof(cnt);
  auto put = [&](const void* src, size_t bytes) {
    if (bytes) std::memcpy(p, src, bytes);
    p += bytes;
  };
  put(d.key.data(), d.key.size() * 8);
  put(d.ptr.data(), d.ptr.size() * 8);
  put(d.col.data(), d.col.size() * 4);
  put(d.val.data(), d.val.size() * 8);
  return IB_OK;
}

ib_status ib_import_operator(ib_solver* s, const void* buf, int64_t size) {
  if (check(s) || !buf || size < 40) return IB_ERR_ARG;
  if (s->prepared) return IB_ERR_STATE;
  const char* p = static_cast<const char*>(buf);
  if (std::memcmp(p, "IBOP0001", 8) != 0) return IB_ERR_ARG;
  int64_t cnt[4];
  std::memcpy(cnt, p + 8, sizeof(cnt));
  for (int k = 0; k < 4; ++k)
    if (cnt[k] < 0 || cnt[k] > size) return IB_ERR_ARG;
  const int64_t need = 40 + cnt[0] * 8 + cnt[1] * 8 + cnt[2] * 4 + cnt[3] * 8;
  if (need != size) return IB_ERR_ARG;
  auto d = std::make_shared<OpData>();
  const char* q = p + 40;
  d->key.resize(cnt[0]);
  d->ptr.resize(cnt[1]);
  d->col.resize(cnt[2]);
  d->val.resize(cnt[3]);
  auto get = [&](void* dst, size_t bytes) {
    if (bytes) std::memcpy(dst, q, bytes);
    q += bytes;
  };
  get(d->key.data(), cnt[0] * 8);
  get(d->ptr.data(), cnt[1] * 8);
  get(d->col.data(), cnt[2] * 4);
  get(d->val.data(), cnt[3] * 8);
  // CSR consistency: monotone row pointers ending at the entry count
  if (!d->ptr.empty()) {
    if (d->ptr.front() != 0 || d->ptr.back() != cnt[2] || cnt[2] != cnt[3]) return IB_ERR_ARG;
    for (size_t k = 1; k < d->ptr.size(); ++k)
      if (d->ptr[k] < d->ptr[k - 1]) return IB_ERR_ARG;
  }
  s->imported = d;
  return IB_OK;
}

ib_status ib_set_operator_cache(int64_t limit_bytes) {
  if (limit_bytes < 0) return IB_ERR_ARG;
  OpCache& c = op_cache();
  std::lock_guard<std::mutex> lk(c.mu);
  c.limit = (size_t)limit_bytes;
  while (c.bytes > c.limit && !c.lru.empty()) {
    c.bytes -= c.lru.back()->bytes();
    c.lru.pop_back();
  }
  return IB_OK;
}

ib_status ib_destroy(ib_solver* s) {
  HipShared hip_lock;
  if (!s) return IB_ERR_ARG;
  if (s->allocated) (void)hipStreamSynchronize(s->stream);
  if (s->side) (void)hipStreamSynchronize(s->side);
  destroy_graphs(s);
  harvest_events(s);
  for (auto e : s->event_pool) (void)hipEventDestroy(e);
  s->event_pool.clear();
  while (!s->allocs.empty()) dfree(s, s->allocs.back().first);
  if (s->hctl) (void)hipHostFree(s->hctl);
  if (s->hpose) (void)hipHostFree(s->hpose);
  if (s->ctl_ready) (void)hipEventDestroy(s->ctl_ready);
  if (s->side) (void)hipStreamDestroy(s->side);
  if (s->l1_done) (void)hipEventDestroy(s->l1_done);
  if (s->side_done) (void)hipEventDestroy(s->side_done);
  delete s;
  return IB_OK;
}

ib_status ib_op_solve(int32_t n, int32_t precision, double alpha, const void* in, void* out,
                      int32_t pitch, void* hip_stream) {
  HipShared hip_lock;
  if (!supported_n(n) || !in || !out || pitch < n - 1 ||
      (precision != IB_FP64 && precision != IB_FP32_FLOW) ||
      (precision == IB_FP64 && !supported_n_fp64(n)))
    return IB_ERR_ARG;
  ib_solver tmp;
  ib_solver* s = &tmp;
  s->stream = static_cast<hipStream_t>(hip_stream);
  s->n = n;
  s->pitch = pitch;
  ib_status st = IB_OK;
  if (precision == IB_FP64) {
    st = make_tables<double>(s, n, &s->tw, &s->lam);
    if (!st) st = op_solve_run<double>(n, pitch, s->stream, alpha, in, out, s->tw, s->lam);
  } else {
    st = make_tables<float>(s, n, &s->tw, &s->lam);
    if (!st) st = op_solve_run<float>(n, pitch, s->stream, alpha, in, out, s->tw, s->lam);
  }
  (void)hipStreamSynchronize(s->stream);
  while (!s->allocs.empty()) dfree(s, s->allocs.back().first);
  return st;
}

ib_status ib_op_solve_noalloc(int32_t n, int32_t precision, double alpha, const void* in,
                              void* out, int32_t pitch, void* hip_stream) {
  HipShared hip_lock;
  if (!supported_n(n) || !in || !out || pitch < n - 1 ||
      (precision != IB_FP64 && precision != IB_FP32_FLOW) ||
      (precision == IB_FP64 && !supported_n_fp64(n)))
    return IB_ERR_ARG;
  hipStream_t st = static_cast<hipStream_t>(hip_stream);
  if (precision == IB_FP64) return op_solve_noalloc_run<double>(n, pitch, st, alpha, in, out);
  return op_solve_noalloc_run<float>(n, pitch, st, alpha, in, out);
}

}  // extern "C"
