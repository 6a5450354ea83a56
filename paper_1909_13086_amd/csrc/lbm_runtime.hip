// Host runtime and C ABI of the B-TriRT melting library (see include/lbm.h).
//
// A context owns one HIP stream (its own or one lent by the caller, e.g. the
// current PyTorch stream), a table of resident cavities ("slots"), an HBM
// budget for admission, reduction scratch and the captured step graphs.  All
// device work is stream-ordered; only the calls that return data block.
#include "lbm.h"
#include "lbm_internal.h"

#include <dlfcn.h>

#include <algorithm>
#include <chrono>
#include <climits>
#include <cstdint>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <fstream>
#include <map>
#include <sstream>
#include <string>
#include <vector>

using lbm::BatchTile;
using lbm::CavDev;
using lbm::LaunchCfg;
using lbm::StatsDev;

namespace {

thread_local std::string g_last_error;

int fail(int code, const std::string &msg) {
  g_last_error = msg;
  return code;
}

#define HIP_TRY(expr)                                                                   \
  do {                                                                                  \
    hipError_t e_ = (expr);                                                             \
    if (e_ != hipSuccess)                                                               \
      return fail(LBM_EDEVICE, std::string(#expr) + ": " + hipGetErrorString(e_));      \
  } while (0)

// Device staging of lbm_fields_noalloc: fixed file-scope device memory, one
// copy on every GPU the library runs on, held until the process ends.  Host
// code reaches it only through the address hipGetSymbolAddress returns for the
// current device (lbm_create keeps it in the context); the array's name in
// host code is not a device address.
constexpr size_t kNoAllocBytes = size_t(16) << 20;
static __device__ __align__(256) unsigned char noalloc_scratch[kNoAllocBytes];

constexpr double kCs2 = 1.0 / 3.0;
constexpr int kPitchAlign = 64;  // cells: one wavefront per row segment
constexpr size_t kByteAlign = 256;

size_t round_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

// Named ranges for ROCm's tracer (roctx): each host call that enqueues or
// waits for GPU work opens one, so `rocprofv3 --marker-trace` shows which
// kernels a call issued.  The roctx library is looked up once at run time;
// without it the ranges cost nothing.
struct Roctx {
  int (*push)(const char *) = nullptr;
  int (*pop)() = nullptr;
};

const Roctx &roctx() {
  static const Roctx r = [] {
    Roctx x;
    void *h = dlopen("librocprofiler-sdk-roctx.so.1", RTLD_NOW | RTLD_LOCAL);
    if (h) {
      x.push = reinterpret_cast<int (*)(const char *)>(dlsym(h, "roctxRangePushA"));
      x.pop = reinterpret_cast<int (*)()>(dlsym(h, "roctxRangePop"));
      if (!x.push || !x.pop) x.push = nullptr, x.pop = nullptr;
    }
    return x;
  }();
  return r;
}

class TraceRange {
 public:
  explicit TraceRange(const char *name) : on_(roctx().push != nullptr) {
    if (on_) roctx().push(name);
  }
  ~TraceRange() {
    if (on_) roctx().pop();
  }
  TraceRange(const TraceRange &) = delete;
  TraceRange &operator=(const TraceRange &) = delete;

 private:
  bool on_;
};

bool rate_ok(double k) { return std::isfinite(k) && k > 0.0 && k < 2.0; }

// Parameter derivation.  Dimensionless mode (reading of Sec. 3.2): the cavity
// height ny is the length scale, Ra = g beta dT ny^3/(nu alpha), Pr = nu/alpha,
// the free-fall velocity sqrt(g beta dT ny) equals Ma*cs, Ste = Cp dT / L.
// Eq. (4): 1/k1 = alpha/cs^2 + 1/2; Eq. (5): k2 = 2 - k1 unless given.  The
// flow's stress moment carries the viscosity the same way.
static_assert(lbm::kSolidScale == LBM_SOLID_SCALE && lbm::kSolidDarcy == LBM_SOLID_DARCY &&
                  lbm::kSolidPbb == LBM_SOLID_PBB,
              "solid model codes");

int derive(const lbm_case *cs, lbm_lattice *out, std::string &why) {
  std::memset(out, 0, sizeof(*out));
  if (!cs) { why = "case is NULL"; return LBM_EINVAL; }
  if (cs->nx < 1 || cs->ny < 1 || cs->nx > (1 << 20) || cs->ny > (1 << 20) ||
      (double)cs->nx * cs->ny > 2.0e9) {
    why = "nx, ny must be >= 1 and the lattice at most 2e9 cells";
    return LBM_EINVAL;
  }
  if (cs->precision != LBM_FP64 && cs->precision != LBM_FP32_SHIFTED) {
    why = "unknown precision"; return LBM_EINVAL;
  }
  if (cs->pattern != LBM_PATTERN_AA && cs->pattern != LBM_PATTERN_AB) {
    why = "unknown streaming pattern"; return LBM_EINVAL;
  }
  if (cs->init < LBM_INIT_SOLID_AT_TM || cs->init > LBM_INIT_GAUSSIAN) {
    why = "unknown initial state"; return LBM_EINVAL;
  }
  if (!(cs->Cp > 0.0) || !(cs->rho0 > 0.0) || !std::isfinite(cs->Cp) ||
      !std::isfinite(cs->rho0) || !std::isfinite(cs->Th) || !std::isfinite(cs->Tm)) {
    why = "Cp and rho0 must be positive, Th and Tm finite"; return LBM_EINVAL;
  }
  const double dT = cs->Th - cs->Tm;
  if (cs->param_mode == LBM_PARAM_DIMENSIONLESS) {
    if (!(cs->Ra > 0.0) || !(cs->Pr > 0.0) || !(cs->Ste > 0.0) || !(cs->Ma > 0.0) ||
        !std::isfinite(cs->Ra) || !std::isfinite(cs->Pr) || !std::isfinite(cs->Ste) ||
        !std::isfinite(cs->Ma)) {
      why = "Ra, Pr, Ste and Ma must be positive"; return LBM_EINVAL;
    }
    if (!(dT > 0.0)) { why = "Th must exceed Tm"; return LBM_EINVAL; }
    const double U = cs->Ma * std::sqrt(kCs2);
    const double ell = (double)cs->ny;
    out->nu = U * ell * std::sqrt(cs->Pr / cs->Ra);
    out->alpha = out->nu / cs->Pr;
    out->gbeta = U * U / (ell * dT);
    out->latent = cs->Cp * dT / cs->Ste;
  } else if (cs->param_mode == LBM_PARAM_LATTICE) {
    out->nu = cs->nu;
    out->alpha = cs->alpha;
    out->gbeta = cs->gbeta;
    out->latent = cs->latent;
  } else {
    why = "unknown parameter mode"; return LBM_EINVAL;
  }
  if (!(out->nu > 0.0) || !(out->alpha > 0.0) || !std::isfinite(out->nu) ||
      !std::isfinite(out->alpha) || !std::isfinite(out->gbeta) || !(out->latent >= 0.0) ||
      !std::isfinite(out->latent)) {
    why = "viscosity and diffusivity must be positive, latent heat >= 0"; return LBM_EINVAL;
  }
  out->k1_g = 1.0 / (out->alpha / kCs2 + 0.5);
  out->k2_g = std::isnan(cs->k2_g) ? 2.0 - out->k1_g : cs->k2_g;
  out->k0_g = std::isnan(cs->k0_g) ? 1.0 : cs->k0_g;
  out->k2_f = 1.0 / (out->nu / kCs2 + 0.5);
  out->k0_f = std::isnan(cs->k0_f) ? 1.0 : cs->k0_f;
  out->k1_f = std::isnan(cs->k1_f) ? 1.0 : cs->k1_f;
  if (!rate_ok(out->k0_g) || !rate_ok(out->k1_g) || !rate_ok(out->k2_g) ||
      !rate_ok(out->k0_f) || !rate_ok(out->k1_f) || !rate_ok(out->k2_f)) {
    why = "every relaxation rate must lie in (0, 2)"; return LBM_EINVAL;
  }
  if (!std::isfinite(cs->heater_center) || !std::isfinite(cs->heater_width)) {
    why = "heater centre and width must be finite"; return LBM_EINVAL;
  }
  // Strip of Sec. 3.2 on cell-centred nodes: cell x is heated when its centre
  // x + 1/2 lies in [(C - D/2) nx, (C + D/2) nx].
  out->heater_lo = 1;
  out->heater_hi = 0;
  if (cs->heater_width > 0.0 && !cs->periodic_y) {
    const double a = (cs->heater_center - 0.5 * cs->heater_width) * cs->nx;
    const double b = (cs->heater_center + 0.5 * cs->heater_width) * cs->nx;
    const double lo = std::max(0.0, std::ceil(a - 0.5));
    const double hi = std::min((double)(cs->nx - 1), std::floor(b - 0.5));
    if (lo <= hi) {
      out->heater_lo = (int32_t)lo;
      out->heater_hi = (int32_t)hi;
    }
  }
  out->n_heater = out->heater_hi >= out->heater_lo ? out->heater_hi - out->heater_lo + 1 : 0;
  if (cs->solid_model < LBM_SOLID_SCALE || cs->solid_model > LBM_SOLID_PBB) {
    why = "unknown solid model"; return LBM_EINVAL;
  }
  out->darcy_c = std::isnan(cs->darcy_c) ? 1e3 : cs->darcy_c;
  out->darcy_eps = std::isnan(cs->darcy_eps) ? 1e-3 : cs->darcy_eps;
  if (!(out->darcy_c >= 0.0) || !std::isfinite(out->darcy_c) || !(out->darcy_eps > 0.0) ||
      !std::isfinite(out->darcy_eps)) {
    why = "Darcy constant must be >= 0 and eps > 0"; return LBM_EINVAL;
  }
  if (cs->init == LBM_INIT_LIQUID_T0 && !std::isfinite(cs->T0)) {
    why = "T0 must be finite"; return LBM_EINVAL;
  }
  if (cs->init == LBM_INIT_GAUSSIAN &&
      (!std::isfinite(cs->T0) || !std::isfinite(cs->gauss_amp) || !(cs->gauss_sigma > 0.0))) {
    why = "Gaussian initial state needs finite T0, amplitude and sigma > 0"; return LBM_EINVAL;
  }
  out->pitch = (int32_t)round_up((size_t)cs->nx, kPitchAlign);
  return LBM_OK;
}

struct Layout {
  size_t pop_bytes;   // one lattice (18 planes)
  size_t cumq_off, cumq_bytes;
  size_t aux_off;     // diagnostics of the state at load (reference enthalpy)
  size_t total;
};

Layout layout_of(const lbm_case *cs, const lbm_lattice &lat) {
  Layout L{};
  const size_t elem = cs->precision == LBM_FP64 ? 8 : 4;
  L.pop_bytes = round_up((size_t)lbm::kPlanes * lat.pitch * (size_t)cs->ny * elem, kByteAlign);
  const size_t lattices = cs->pattern == LBM_PATTERN_AB ? 2 : 1;
  L.cumq_off = lattices * L.pop_bytes;
  L.cumq_bytes = round_up((size_t)cs->nx * sizeof(double), kByteAlign);
  L.aux_off = L.cumq_off + L.cumq_bytes;
  L.total = L.aux_off + round_up(sizeof(StatsDev), kByteAlign);
  return L;
}

struct Slot {
  bool used = false;
  lbm_case cs{};
  lbm_lattice lat{};
  Layout lay{};
  CavDev dev{};
  void *base = nullptr;
  bool owned = false;
  int64_t step = 0;
  StatsDev *e0_dev = nullptr;  // diagnostics of the state at load, on the device
  // diagnostics recorded during lbm_step
  int64_t report_every = 0;
  int32_t report_cap = 0;
  StatsDev *series = nullptr;
  std::vector<int64_t> series_step;
  std::vector<int32_t> series_parity;
  // captured step chunks, keyed by starting parity
  hipGraphExec_t graph[2] = {nullptr, nullptr};
  int graph_after[2] = {0, 1};  // storage parity after a replay
  int graph_chunk = 0;
};

// Batched execution.  Resident cavities are packed into cache groups whose
// summed footprint fits the last-level (Infinity) cache; within a chunk every
// group advances all its steps before the next group starts, so after its
// first step a group's populations are served from that cache.  Groups are
// independent cavities, so the order changes no result.
struct Batch {
  CavDev *cavs_dev = nullptr;
  BatchTile *tiles_dev = nullptr;
  int32_t *hdr_dev = nullptr;     // per (group, precision): {first tile, tile count}
  size_t cav_cap = 0, tile_cap = 0, hdr_cap = 0;
  CavDev *cavs_host = nullptr;    // pinned staging
  BatchTile *tiles_host = nullptr;
  int32_t *hdr_host = nullptr;
  std::vector<int> members;       // slot ids in cavity-array order
  std::vector<int> group_precs;   // per group: bit launch_bit(p, kind, model) set when it holds
                                  // such launches (kind 0: one step per launch over tiles,
                                  // kind 1 / 2: two- / three-step launches over strip segments)
  std::vector<int> hdr_seg;       // per header: segment rows of its fused launches
  bool dirty = true;
  hipGraphExec_t graph = nullptr; // valid while the device buffers and the group shape stay
  int graph_chunk = 0;
  std::vector<int> graph_shape;   // group_precs the graph was captured for
  std::vector<int> graph_segs;    // hdr_seg the graph was captured for
};

}  // namespace

void lbm::set_last_error(const std::string &msg) { g_last_error = msg; }

struct lbm_ctx {
  int device = 0;
  hipStream_t stream = nullptr;
  bool own_stream = false;
  size_t budget = 0, used = 0;
  std::vector<Slot> slots;
  double *partials = nullptr;
  int32_t *err_dev = nullptr;      // device error word of the batched kernels (kErrBatchHeader)
  int32_t *err_host = nullptr;     // pinned copy, read after the stream has drained
  StatsDev *stats_dev = nullptr;
  StatsDev *stats_host = nullptr;  // pinned, 2 entries: current state and state at load
  void *scratch = nullptr;
  size_t scratch_bytes = 0;
  void *noalloc = nullptr;         // this device's copy of noalloc_scratch (kNoAllocBytes)
  LaunchCfg launch[2] = {lbm::default_launch(0), lbm::default_launch(1)};
  int graph_chunk = 0;
  int num_cus = 256;
  // resident wavefronts per CU of the fused single-cavity kernels, per
  // [precision][steps per launch][kernel variant][rows staged] (lbm_create)
  int fused_wpc[2][5][lbm::kKernelModels][2] = {};
  size_t group_bytes = size_t(192) << 20;  // cache-group capacity of the batched launch
  Batch batch;
};

namespace {

int check_slot(lbm_ctx *c, int slot) {
  if (!c) return fail(LBM_EINVAL, "context is NULL");
  if (slot < 0 || slot >= (int)c->slots.size() || !c->slots[slot].used)
    return fail(LBM_ESTATE, "slot " + std::to_string(slot) + " is not in use");
  return LBM_OK;
}

// Copies the device error word behind the work already enqueued (no wait).
hipError_t enqueue_error_copy(lbm_ctx *c) {
  return hipMemcpyAsync(c->err_host, c->err_dev, sizeof(int32_t), hipMemcpyDeviceToHost, c->stream);
}

// After the stream has drained past an enqueue_error_copy: turns a device error
// raised by a batched kernel into LBM_EDEVICE and clears the word.
int take_device_error(lbm_ctx *c) {
  const int32_t e = *c->err_host;
  if (e == 0) return LBM_OK;
  *c->err_host = 0;
  HIP_TRY(lbm::launch_fill_zero(c->err_dev, sizeof(int32_t), c->stream));
  HIP_TRY(hipStreamSynchronize(c->stream));
  return fail(LBM_EDEVICE, "a batched launch found its work-list header empty or out of range "
                           "and advanced nothing (code " + std::to_string(e) + ")");
}

// Waits for the stream and reports a device error raised since the last check.
int sync_checked(lbm_ctx *c) {
  HIP_TRY(enqueue_error_copy(c));
  HIP_TRY(hipStreamSynchronize(c->stream));
  return take_device_error(c);
}

int ensure_scratch(lbm_ctx *c, size_t bytes) {
  if (bytes <= c->scratch_bytes) return LBM_OK;
  if (c->scratch) {
    HIP_TRY(hipStreamSynchronize(c->stream));
    HIP_TRY(hipFree(c->scratch));
    c->scratch = nullptr;
    c->scratch_bytes = 0;
  }
  const size_t want = round_up(bytes, 1 << 20);
  if (hipMalloc(&c->scratch, want) != hipSuccess) {
    c->scratch = nullptr;
    (void)hipGetLastError();
    return fail(LBM_ENOMEM, "cannot allocate " + std::to_string(want) + " bytes of scratch");
  }
  c->scratch_bytes = want;
  return LBM_OK;
}

void drop_graphs(Slot &s) {
  for (auto &g : s.graph) {
    if (g) (void)hipGraphExecDestroy(g);
    g = nullptr;
  }
  s.graph_chunk = 0;
}

void drop_batch_graph(lbm_ctx *c) {
  if (c->batch.graph) (void)hipGraphExecDestroy(c->batch.graph);
  c->batch.graph = nullptr;
  c->batch.graph_chunk = 0;
}

CavDev make_dev(const lbm_case *cs, const lbm_lattice &lat, const Layout &lay, void *base) {
  CavDev d{};
  d.nx = cs->nx;
  d.ny = cs->ny;
  d.pitch = lat.pitch;
  d.periodic_x = cs->periodic_x != 0;
  d.periodic_y = cs->periodic_y != 0;
  d.hlo = lat.heater_lo;
  d.hhi = lat.heater_hi;
  d.parity = 0;
  d.pattern = cs->pattern;
  d.active_steps = 0;
  d.solid_model = cs->solid_model;
  d.darcy_c = lat.darcy_c;
  d.darcy_eps = lat.darcy_eps;
  d.plane = lbm::kWave;  // blocked layout: planes of a 64-cell chunk are 64 elements apart
  d.k0g = lat.k0_g;
  d.k1g = lat.k1_g;
  d.k2g = lat.k2_g;
  d.k0f = lat.k0_f;
  d.k1f = lat.k1_f;
  d.k2f = lat.k2_f;
  d.Cp = cs->Cp;
  d.inv_Cp = 1.0 / cs->Cp;
  d.latent = lat.latent;
  d.inv_latent = lat.latent > 0.0 ? 1.0 / lat.latent : 0.0;
  d.rho0 = cs->rho0;
  d.inv_rho0 = 1.0 / cs->rho0;
  d.gbeta_rho0 = cs->rho0 * lat.gbeta;
  d.dT = cs->Th - cs->Tm;
  d.Tm = cs->Tm;
  d.alpha = lat.alpha;
  char *b = static_cast<char *>(base);
  d.pop[0] = b;
  d.pop[1] = cs->pattern == LBM_PATTERN_AB ? b + lay.pop_bytes : nullptr;
  d.cumq = reinterpret_cast<double *>(b + lay.cumq_off);
  set_rates(d);
  return d;
}

// Diagnostics of the current state; *e0 gets the total enthalpy at load.
int reduce_now(lbm_ctx *c, Slot &s, StatsDev *out_host, double *e0) {
  HIP_TRY(lbm::launch_reduce(s.dev, s.cs.precision, c->partials, c->stats_dev, c->stream));
  HIP_TRY(hipMemcpyAsync(c->stats_host, c->stats_dev, sizeof(StatsDev), hipMemcpyDeviceToHost,
                         c->stream));
  HIP_TRY(hipMemcpyAsync(c->stats_host + 1, s.e0_dev, sizeof(StatsDev), hipMemcpyDeviceToHost,
                         c->stream));
  const int rc = sync_checked(c);
  if (rc != LBM_OK) return rc;
  *out_host = c->stats_host[0];
  *e0 = c->stats_host[1].total_H;
  return LBM_OK;
}

void fill_stats(const Slot &s, const StatsDev &d, double E0, int64_t step, int32_t parity,
                lbm_stats *o) {
  std::memset(o, 0, sizeof(*o));
  o->step = step;
  o->melt_fraction = d.melt_fraction;
  o->heater_q = d.heater_q;
  const double dT = s.cs.Th - s.cs.Tm;
  o->nusselt = (s.lat.n_heater > 0 && dT != 0.0)
                   ? (double)s.cs.ny * d.heater_q / ((double)s.lat.n_heater * s.lat.alpha * s.cs.Cp * dT)
                   : 0.0;
  o->total_H = d.total_H;
  o->heat_in_cum = d.heat_in_cum;
  o->budget_residual = d.total_H - E0 - d.heat_in_cum;
  o->mass = d.mass;
  o->max_u = d.max_u;
  o->fourier = s.lat.alpha * (double)step / ((double)s.cs.ny * (double)s.cs.ny);
  o->finite = d.nonfinite == 0.0 ? 1 : 0;
  o->parity = parity;
}

// Resets step counter and strip budget after a new state and records the
// state's diagnostics on the device as the budget reference (stream-ordered,
// no wait).
int restart_clock(lbm_ctx *c, Slot &s) {
  HIP_TRY(lbm::launch_fill_zero(s.dev.cumq, s.lay.cumq_bytes, c->stream));
  s.step = 0;
  s.series_step.clear();
  s.series_parity.clear();
  HIP_TRY(lbm::launch_reduce(s.dev, s.cs.precision, c->partials, s.e0_dev, c->stream));
  return LBM_OK;
}

int enqueue_one_step(lbm_ctx *c, Slot &s) {
  HIP_TRY(lbm::launch_step(s.dev, s.cs.precision, c->launch[s.cs.precision], c->stream));
  s.dev.parity ^= 1;
  s.step += 1;
  return LBM_OK;
}

// Segment rows of a single-cavity launch fusing `steps` steps over strips of
// the given count, under the default fusion.  When some length lets every
// wavefront of the launch be resident at once (`slots` of them: one pass),
// the rows minimise the modelled time
//   passes x rows collided per segment x max(rho, resident waves per SIMD),
// rows collided being steps x rows stored plus steps (steps - 1) halo rows:
// a wavefront's walk costs its rows either in latency (rho, the latency of a
// row over its arithmetic on one SIMD) or, with more waves per SIMD than
// that, in shared arithmetic.  Short segments so fill the launch of a small
// cavity, and a one-pass length spares a larger one an idle tail pass.
// Otherwise (many passes) the configured rows stand, which measured best on
// the large cavities.
int pick_rows(int64_t strips, int ny, int steps, int rows, int64_t slots, int64_t simds, double rho) {
  if (slots <= 0 || simds <= 0) return rows;
  int best = rows;
  double best_cost = 1e300;
  bool one_pass = false;
  for (int r : {1, 2, 3, 4, 6, 8}) {
    const int64_t waves = strips * ((ny + r - 1) / r);
    const int64_t passes = (waves + slots - 1) / slots;
    one_pass = one_pass || passes == 1;
    const double per_simd = (double)std::min(waves, slots) / (double)simds;
    const double cost = (double)passes * (steps * r + steps * (steps - 1)) * std::max(rho, per_simd);
    if (cost < best_cost) {
      best_cost = cost;
      best = r;
    }
  }
  return one_pass ? best : rows;
}

// The launch configuration of one slot.  Unless the context's fusion is set
// explicitly (by lbm_set_fusion or lbm_autotune) it follows the cavity size,
// as measured on MI355X: FP64 cavities below 2^18 cells take two steps per
// launch (the three-step kernel wins only on larger ones), FP32 cavities of
// 2^21 cells or more take four (below, where the lattices sit in the
// Infinity Cache, three are faster), and the segment rows follow pick_rows
// with the resident wavefronts of the kernel the launch uses.
LaunchCfg slot_launch(const lbm_ctx *c, const Slot &s) {
  LaunchCfg L = c->launch[s.cs.precision];
  if (!L.adapt || s.cs.pattern != LBM_PATTERN_AB) return L;
  const int64_t cells = (int64_t)s.cs.nx * s.cs.ny;
  if (L.fuse == 3 && s.cs.precision == LBM_FP64 && cells < (int64_t)1 << 18) L.fuse = 2;
  if (L.fuse == 3 && s.cs.precision == LBM_FP32_SHIFTED && cells >= (int64_t)1 << 21) L.fuse = 4;
  if (L.fuse >= 2) {
    const int cols = L.fuse == 2 ? lbm::kStripCols : (L.fuse == 3 ? lbm::kStrip3Cols : lbm::kStrip4Cols);
    int &rows = L.fuse == 2 ? L.seg : (L.fuse == 3 ? L.seg3 : L.seg4);
    const int wpc = c->fused_wpc[s.cs.precision][L.fuse][s.dev.kmodel][L.staged ? 1 : 0];
    // rho as fitted on MI355X: the FP64 walks are bound by row latency at any
    // residency they reach (2 waves per SIMD), the FP32 ones, whose rows carry
    // the same arithmetic on half the bytes, by arithmetic above 1.5 waves
    const double rho = s.cs.precision == LBM_FP64 ? 4.0 : 1.5;
    rows = pick_rows((s.cs.nx + cols - 1) / cols, s.cs.ny, L.fuse, rows, (int64_t)wpc * c->num_cus,
                     (int64_t)4 * c->num_cus /* four SIMDs per CU */, rho);
  }
  return L;
}

// Steps per launch of a slot: two-lattice slots may advance two, three or
// (FP32) four steps per launch, in-place slots one.
int steps_per_launch(const lbm_ctx *c, const Slot &s) {
  return s.cs.pattern == LBM_PATTERN_AB ? slot_launch(c, s).fuse : 1;
}

// One launch advancing the state by m steps (1 to 4, at most the slot's
// steps per launch).  Every launch moves the state to the other lattice of a
// two-lattice slot; in place it flips the A-A parity.
hipError_t launch_steps(const lbm_ctx *c, const Slot &s, const CavDev &d, int m) {
  const LaunchCfg L = slot_launch(c, s);
  if (m == 4) return lbm::launch_step4(d, s.cs.precision, L, c->stream);
  if (m == 3) return lbm::launch_step3(d, s.cs.precision, L, c->stream);
  if (m == 2) return lbm::launch_step2(d, s.cs.precision, L, c->stream);
  return lbm::launch_step(d, s.cs.precision, L, c->stream);
}

int enqueue_steps(lbm_ctx *c, Slot &s, int m) {
  HIP_TRY(launch_steps(c, s, s.dev, m));
  s.dev.parity ^= 1;
  s.step += m;
  return LBM_OK;
}

// Steps of the next launch when `left` steps remain before the next stop
// (a report or the end of the request): the slot's steps per launch, fewer
// at the end, and one fewer when one more than that remains, so that no
// single step is left over (four steps as two and two, five as three and
// two: two fused launches cost less than a deep one and a single step).
int64_t next_launch_steps(int F, int64_t left) {
  if (F >= 3 && left == F + 1) return F - 1;
  return std::min<int64_t>(F, left);
}

// Launches of a chunk of n steps starting from parity p (next_launch_steps).
// Returns the storage parity after the chunk.
int enqueue_chunk(lbm_ctx *c, const Slot &s, CavDev d, int n, hipError_t *err) {
  const int F = steps_per_launch(c, s);
  *err = hipSuccess;
  for (int k = 0; k < n && *err == hipSuccess;) {
    const int m = (int)next_launch_steps(F, n - k);
    *err = launch_steps(c, s, d, m);
    d.parity ^= 1;
    k += m;
  }
  return d.parity;
}

int record_report(lbm_ctx *c, Slot &s) {
  if (s.report_every <= 0 || s.step % s.report_every != 0) return LBM_OK;
  const int32_t k = (int32_t)s.series_step.size();
  if (k >= s.report_cap) return LBM_OK;
  HIP_TRY(lbm::launch_reduce(s.dev, s.cs.precision, c->partials, s.series + k, c->stream));
  s.series_step.push_back(s.step);
  s.series_parity.push_back(s.dev.parity);
  return LBM_OK;
}

// Captures a chunk of steps starting at storage parity p.
int capture_chunk(lbm_ctx *c, Slot &s, int p, int chunk) {
  CavDev d = s.dev;
  d.parity = p;
  hipGraph_t g = nullptr;
  HIP_TRY(hipStreamBeginCapture(c->stream, hipStreamCaptureModeThreadLocal));
  hipError_t err = hipSuccess;
  const int after = enqueue_chunk(c, s, d, chunk, &err);
  hipError_t e2 = hipStreamEndCapture(c->stream, &g);
  if (err != hipSuccess || e2 != hipSuccess) {
    if (g) (void)hipGraphDestroy(g);
    return fail(LBM_EDEVICE, std::string("graph capture: ") +
                                 hipGetErrorString(err != hipSuccess ? err : e2));
  }
  hipGraphExec_t ex = nullptr;
  hipError_t e3 = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
  (void)hipGraphDestroy(g);
  if (e3 != hipSuccess) return fail(LBM_EDEVICE, std::string("graph instantiate: ") + hipGetErrorString(e3));
  s.graph[p] = ex;
  s.graph_after[p] = after;
  return LBM_OK;
}

int step_slot(lbm_ctx *c, Slot &s, int64_t n) {
  const int chunk = c->graph_chunk;
  if (chunk != s.graph_chunk) {
    drop_graphs(s);
    s.graph_chunk = chunk;
  }
  while (n > 0) {
    // graph replay only when no report falls strictly inside the chunk
    bool use_graph = chunk > 0 && n >= chunk;
    const int64_t next =
        s.report_every > 0 ? (s.step / s.report_every + 1) * s.report_every : INT64_MAX;
    if (use_graph && next < s.step + chunk) use_graph = false;
    int rc = LBM_OK;
    if (use_graph) {
      const int p = s.dev.parity;
      if (!s.graph[p]) {
        rc = capture_chunk(c, s, p, chunk);
        if (rc != LBM_OK) return rc;
      }
      HIP_TRY(hipGraphLaunch(s.graph[p], c->stream));
      s.step += chunk;
      s.dev.parity = s.graph_after[p];
      n -= chunk;
    } else {
      // as many fused steps as fit before the next report
      const int64_t m = next_launch_steps(steps_per_launch(c, s), std::min<int64_t>(n, next - s.step));
      rc = m >= 2 ? enqueue_steps(c, s, (int)m) : enqueue_one_step(c, s);
      n -= m >= 2 ? m : 1;
    }
    if (rc != LBM_OK) return rc;
    rc = record_report(c, s);
    if (rc != LBM_OK) return rc;
  }
  return LBM_OK;
}

}  // namespace

// ---------------------------------------------------------------------------
// batched launch over every resident slot

namespace {

constexpr int kBatchTileX = 64;
constexpr int kBatchTileRows = 16;
constexpr int kStrip2Cols = lbm::kStripCols;

// Launches of a cache group come per precision, kind (one-step tiles, two-
// or three-step segments) and kernel variant (solid model, or the scaled
// model with k0 = 1: CavDev::kmodel); each has a {first, count} header.
constexpr int kLaunchKinds = 2 * 3 * lbm::kKernelModels;
static_assert(kLaunchKinds <= 31, "launch kinds are bits of an int");
int launch_bit(int prec, int kind, int model) { return (prec * 3 + kind) * lbm::kKernelModels + model; }
// kind of a slot's batched launches: its steps per launch - 1 (batched
// launches fuse at most three steps; a four-step slot takes three there)
int batch_kind(const lbm_ctx *c, const Slot &s) { return std::min(steps_per_launch(c, s), 3) - 1; }
// kernel variant a slot's batched launches of the given kind use: the
// one-step tiles keep the general collision, so their unit-k0 cavities share
// the launch of the scaled model
int batch_model(const Slot &s, int kind) {
  return kind == 0 && s.dev.kmodel == lbm::kScaleUnitK0 ? lbm::kSolidScale : s.dev.kmodel;
}
int hdr_index(int g, int prec, int kind, int model) {
  return (g * kLaunchKinds + launch_bit(prec, kind, model)) * 2;
}

void free_batch(lbm_ctx *c) {
  Batch &b = c->batch;
  drop_batch_graph(c);
  if (b.cavs_dev) (void)hipFree(b.cavs_dev);
  if (b.tiles_dev) (void)hipFree(b.tiles_dev);
  if (b.hdr_dev) (void)hipFree(b.hdr_dev);
  if (b.cavs_host) (void)hipHostFree(b.cavs_host);
  if (b.tiles_host) (void)hipHostFree(b.tiles_host);
  if (b.hdr_host) (void)hipHostFree(b.hdr_host);
  b.cavs_dev = nullptr;
  b.tiles_dev = nullptr;
  b.hdr_dev = nullptr;
  b.cavs_host = nullptr;
  b.tiles_host = nullptr;
  b.hdr_host = nullptr;
  b.cav_cap = b.tile_cap = b.hdr_cap = 0;
}

// A cavity larger than the cache-group capacity gains nothing from sharing
// launches (it would form a group of its own, too large for the cache); it
// steps on the single-cavity path, whose kernels take the whole device.
bool solo_slot(const lbm_ctx *c, const Slot &s) { return s.lay.total > c->group_bytes; }

// Tile lists of every resident slot that is not solo, grouped by cache group
// then precision.  The device buffers only grow, so a captured graph
// survives membership changes that keep the group shape.
int rebuild_batch(lbm_ctx *c) {
  Batch &b = c->batch;
  b.members.clear();
  for (int i = 0; i < (int)c->slots.size(); ++i)
    if (c->slots[i].used && !solo_slot(c, c->slots[i])) b.members.push_back(i);
  // greedy packing in slot order: a group closes when the next cavity would
  // overflow the capacity
  std::vector<int> group_of(b.members.size(), 0);
  int ngroups = b.members.empty() ? 0 : 1;
  size_t acc = 0;
  for (size_t j = 0; j < b.members.size(); ++j) {
    const size_t fp = c->slots[b.members[j]].lay.total;
    if (acc > 0 && acc + fp > c->group_bytes) {
      ++ngroups;
      acc = 0;
    }
    acc += fp;
    group_of[j] = ngroups - 1;
  }
  const size_t ncav = b.members.size();
  auto cols_of = [](int kind) { return kind == 2 ? lbm::kStrip3Cols : kStrip2Cols; };
  auto segs_of = [](const Slot &s, int cols, int seg) -> int64_t {
    return (int64_t)((s.cs.nx + cols - 1) / cols) * ((s.cs.ny + seg - 1) / seg);
  };
  // Segment rows of each fused launch.  While the fusion is the default they
  // balance the launch: its wavefronts (one per segment) take segments in
  // passes of step2_batch_grid x 2, and a segment of seg rows advanced by
  // kind + 1 steps costs each lane (kind + 1) seg + kind (kind + 1)
  // collisions (the halo rows of every level included), so the rows that
  // minimise passes x cost are taken (a launch of few segments prefers short
  // ones, one just above a full pass longer ones).
  const int64_t wave_slots = (int64_t)lbm::step2_batch_grid(c->num_cus) * 2;
  b.hdr_seg.assign((size_t)std::max(ngroups, 1) * kLaunchKinds, 0);
  for (int g = 0; g < ngroups; ++g)
    for (int prec = 0; prec < 2; ++prec)
      for (int kind = 1; kind < 3; ++kind)
        for (int model = 0; model < lbm::kKernelModels; ++model) {
          const LaunchCfg &L = c->launch[prec];
          int best = kind == 2 ? L.seg3 : L.seg;
          if (L.adapt) {
            double best_cost = 1e300;
            for (int seg = 1; seg <= 16; ++seg) {
              int64_t items = 0;
              for (size_t j = 0; j < ncav; ++j) {
                const Slot &s = c->slots[b.members[j]];
                if (group_of[j] == g && s.cs.precision == prec && batch_kind(c, s) == kind &&
                    batch_model(s, kind) == model)
                  items += segs_of(s, cols_of(kind), seg);
              }
              if (items == 0) break;
              const double cost =
                  (double)((items + wave_slots - 1) / wave_slots) * ((kind + 1) * seg + kind * (kind + 1));
              if (cost < best_cost) {
                best_cost = cost;
                best = seg;
              }
            }
          }
          b.hdr_seg[hdr_index(g, prec, kind, model) / 2] = best;
        }
  // work items: 64 x 16 tiles for one-step cavities, strip segments (62
  // columns for two steps, 60 for three, one wavefront each) for fused ones
  size_t ntiles = 0;
  for (size_t j = 0; j < ncav; ++j) {
    const Slot &s = c->slots[b.members[j]];
    const int kind = batch_kind(c, s);
    if (kind == 0)
      ntiles += (size_t)((s.cs.nx + kBatchTileX - 1) / kBatchTileX) *
                ((s.cs.ny + kBatchTileRows - 1) / kBatchTileRows);
    else
      ntiles += (size_t)segs_of(s, cols_of(kind),
                                b.hdr_seg[hdr_index(group_of[j], s.cs.precision, kind, batch_model(s, kind)) / 2]);
  }
  const size_t nhdr = (size_t)std::max(ngroups, 1) * kLaunchKinds * 2;
  HIP_TRY(hipStreamSynchronize(c->stream));  // staging buffers may feed an earlier copy
  if (ncav > b.cav_cap || ntiles > b.tile_cap || nhdr > b.hdr_cap) {
    free_batch(c);
    b.cav_cap = std::max<size_t>(ncav, c->slots.size());
    b.tile_cap = std::max<size_t>(ntiles * 2, 4096);
    b.hdr_cap = std::max<size_t>(nhdr * 2, (size_t)kLaunchKinds * 2 * 64);
    HIP_TRY(hipMalloc(&b.cavs_dev, b.cav_cap * sizeof(CavDev)));
    HIP_TRY(hipMalloc(&b.tiles_dev, b.tile_cap * sizeof(BatchTile)));
    HIP_TRY(hipMalloc(&b.hdr_dev, b.hdr_cap * sizeof(int32_t)));
    HIP_TRY(hipHostMalloc(&b.cavs_host, b.cav_cap * sizeof(CavDev)));
    HIP_TRY(hipHostMalloc(&b.tiles_host, b.tile_cap * sizeof(BatchTile)));
    HIP_TRY(hipHostMalloc(&b.hdr_host, b.hdr_cap * sizeof(int32_t)));
    HIP_TRY(lbm::launch_fill_zero(b.hdr_dev, b.hdr_cap * sizeof(int32_t), c->stream));
  }
  b.group_precs.assign(ngroups, 0);
  size_t t = 0;
  for (int g = 0; g < ngroups; ++g) {
    for (int prec = 0; prec < 2; ++prec) {
      for (int kind = 0; kind < 3; ++kind) {
        for (int model = 0; model < lbm::kKernelModels; ++model) {
          const size_t first = t;
          for (size_t j = 0; j < ncav; ++j) {
            if (group_of[j] != g) continue;
            const Slot &s = c->slots[b.members[j]];
            if (s.cs.precision != prec || batch_kind(c, s) != kind || batch_model(s, kind) != model)
              continue;
            if (kind == 0) {
              for (int y0 = 0; y0 < s.cs.ny; y0 += kBatchTileRows)
                for (int x0 = 0; x0 < s.cs.nx; x0 += kBatchTileX)
                  b.tiles_host[t++] = BatchTile{(int32_t)j, x0, y0, 0};
            } else {
              const int seg = b.hdr_seg[hdr_index(g, prec, kind, model) / 2];
              const int cols = cols_of(kind);
              for (int y0 = 0, k = 0; y0 < s.cs.ny; y0 += seg, ++k)
                for (int x0 = 0; x0 < s.cs.nx; x0 += cols)
                  b.tiles_host[t++] = BatchTile{(int32_t)j, x0, y0, k};
            }
          }
          const int h = hdr_index(g, prec, kind, model);
          b.hdr_host[h] = (int32_t)first;
          b.hdr_host[h + 1] = (int32_t)(t - first);
          if (t > first) b.group_precs[g] |= 1 << launch_bit(prec, kind, model);
        }
      }
    }
  }
  // every header a launch will read addresses a non-empty range of the list
  for (int g = 0; g < ngroups; ++g)
    for (int bit = 0; bit < kLaunchKinds; ++bit) {
      if (!(b.group_precs[g] & (1 << bit))) continue;
      const int32_t first = b.hdr_host[(g * kLaunchKinds + bit) * 2];
      const int32_t count = b.hdr_host[(g * kLaunchKinds + bit) * 2 + 1];
      if (first < 0 || count <= 0 || (size_t)first + (size_t)count > t || t > b.tile_cap)
        return fail(LBM_ESTATE, "batched work list inconsistent: header {" + std::to_string(first) + ", " +
                                    std::to_string(count) + "} over " + std::to_string(t) + " items");
    }
  if (t > 0)
    HIP_TRY(hipMemcpyAsync(b.tiles_dev, b.tiles_host, t * sizeof(BatchTile),
                           hipMemcpyHostToDevice, c->stream));
  if (ngroups > 0)
    HIP_TRY(hipMemcpyAsync(b.hdr_dev, b.hdr_host,
                           (size_t)ngroups * kLaunchKinds * 2 * sizeof(int32_t),
                           hipMemcpyHostToDevice, c->stream));
  b.dirty = false;
  return LBM_OK;
}

int batch_grid(lbm_ctx *c) { return c->num_cus * 8; }

// Launches of one chunk: per cache group, `chunk` one-step launches,
// ceil(chunk / 2) two-step and ceil(chunk / 3) three-step launches for each
// precision present.
hipError_t enqueue_batch_chunk(lbm_ctx *c, int chunk) {
  Batch &b = c->batch;
  hipError_t err = hipSuccess;
  for (int g = 0; g < (int)b.group_precs.size() && err == hipSuccess; ++g) {
    for (int k = 0; k < chunk && err == hipSuccess; ++k)
      for (int prec = 0; prec < 2 && err == hipSuccess; ++prec)
        for (int model = 0; model < lbm::kKernelModels && err == hipSuccess; ++model)
          if (b.group_precs[g] & (1 << launch_bit(prec, 0, model)))
            err = lbm::launch_step_batch(b.cavs_dev, b.tiles_dev,
                                         b.hdr_dev + hdr_index(g, prec, 0, model), (int)b.tile_cap,
                                         prec, model, kBatchTileX, kBatchTileRows, k,
                                         batch_grid(c), c->err_dev, c->stream);
    for (int j = 0; j < (chunk + 1) / 2 && err == hipSuccess; ++j)
      for (int prec = 0; prec < 2 && err == hipSuccess; ++prec)
        for (int model = 0; model < lbm::kKernelModels && err == hipSuccess; ++model)
          if (b.group_precs[g] & (1 << launch_bit(prec, 1, model))) {
            LaunchCfg L = c->launch[prec];
            L.seg = b.hdr_seg[hdr_index(g, prec, 1, model) / 2];
            err = lbm::launch_step2_batch(b.cavs_dev, b.tiles_dev,
                                          b.hdr_dev + hdr_index(g, prec, 1, model),
                                          (int)b.tile_cap, prec, model, L, j,
                                          lbm::step2_batch_grid(c->num_cus), c->err_dev, c->stream);
          }
    for (int j = 0; j < (chunk + 2) / 3 && err == hipSuccess; ++j)
      for (int prec = 0; prec < 2 && err == hipSuccess; ++prec)
        for (int model = 0; model < lbm::kKernelModels && err == hipSuccess; ++model)
          if (b.group_precs[g] & (1 << launch_bit(prec, 2, model))) {
            LaunchCfg L = c->launch[prec];
            L.seg3 = b.hdr_seg[hdr_index(g, prec, 2, model) / 2];
            err = lbm::launch_step3_batch(b.cavs_dev, b.tiles_dev,
                                          b.hdr_dev + hdr_index(g, prec, 2, model),
                                          (int)b.tile_cap, prec, model, L, j,
                                          lbm::step2_batch_grid(c->num_cus), c->err_dev, c->stream);
          }
  }
  return err;
}

// Advances slot ids[j] by n[j] steps (0 <= n[j]) with batched launches: one
// launch per step per (cache group, precision), chunks of c->graph_chunk
// launches replayed from a captured graph.
int step_many(lbm_ctx *c, const std::vector<int> &ids, const std::vector<int64_t> &n) {
  Batch &b = c->batch;
  if (b.dirty) {
    int rc = rebuild_batch(c);
    if (rc != LBM_OK) return rc;
  }
  std::vector<int64_t> left(c->slots.size(), 0);
  for (size_t j = 0; j < ids.size(); ++j) left[ids[j]] += n[j];
  // solo cavities on the single-cavity path (stream-ordered like the rest)
  for (size_t id = 0; id < left.size(); ++id)
    if (left[id] > 0 && solo_slot(c, c->slots[id])) {
      int rc = step_slot(c, c->slots[id], left[id]);
      if (rc != LBM_OK) return rc;
      left[id] = 0;
    }
  int64_t most = 0;
  for (int64_t v : left) most = std::max(most, v);
  if (most == 0) return LBM_OK;
  // recorded diagnostics need per-step hooks: those slots step on their own
  bool reports = false;
  for (int id : ids) reports = reports || c->slots[id].report_every > 0;
  if (reports) {
    for (size_t id = 0; id < left.size(); ++id)
      if (left[id] > 0) {
        int rc = step_slot(c, c->slots[id], left[id]);
        if (rc != LBM_OK) return rc;
      }
    return LBM_OK;
  }
  const int cap = c->graph_chunk > 0 ? c->graph_chunk : 64;
  while (most > 0) {
    const int chunk = (int)std::min<int64_t>(most, cap);
    {
      // staging buffer reuse; a device error of the previous chunk surfaces here
      const int rc = sync_checked(c);
      if (rc != LBM_OK) return rc;
    }
    for (size_t j = 0; j < b.members.size(); ++j) {
      const int id = b.members[j];
      CavDev d = c->slots[id].dev;
      d.active_steps = (int32_t)std::min<int64_t>(left[id], chunk);
      b.cavs_host[j] = d;
    }
    HIP_TRY(hipMemcpyAsync(b.cavs_dev, b.cavs_host, b.members.size() * sizeof(CavDev),
                           hipMemcpyHostToDevice, c->stream));
    const bool use_graph = c->graph_chunk > 0 && chunk == c->graph_chunk;
    if (use_graph) {
      if (!b.graph || b.graph_chunk != chunk || b.graph_shape != b.group_precs ||
          b.graph_segs != b.hdr_seg) {
        drop_batch_graph(c);
        hipGraph_t g = nullptr;
        HIP_TRY(hipStreamBeginCapture(c->stream, hipStreamCaptureModeThreadLocal));
        hipError_t err = enqueue_batch_chunk(c, chunk);
        hipError_t e2 = hipStreamEndCapture(c->stream, &g);
        if (err != hipSuccess || e2 != hipSuccess) {
          if (g) (void)hipGraphDestroy(g);
          return fail(LBM_EDEVICE, "batched graph capture failed");
        }
        hipError_t e3 = hipGraphInstantiate(&b.graph, g, nullptr, nullptr, 0);
        (void)hipGraphDestroy(g);
        if (e3 != hipSuccess) {
          b.graph = nullptr;
          return fail(LBM_EDEVICE, "batched graph instantiate failed");
        }
        b.graph_chunk = chunk;
        b.graph_shape = b.group_precs;
        b.graph_segs = b.hdr_seg;
      }
      HIP_TRY(hipGraphLaunch(b.graph, c->stream));
    } else {
      HIP_TRY(enqueue_batch_chunk(c, chunk));
    }
    for (int id : b.members) {
      Slot &s = c->slots[id];
      const int64_t adv = std::min<int64_t>(left[id], chunk);
      s.step += adv;
      // one parity flip per launch that advanced the slot
      const int F = batch_kind(c, s) + 1;
      const int64_t launches = (adv + F - 1) / F;
      if (launches & 1) s.dev.parity ^= 1;
      left[id] -= adv;
    }
    most -= chunk;
  }
  HIP_TRY(enqueue_error_copy(c));
  return LBM_OK;
}

int step_all(lbm_ctx *c, int64_t n) {
  std::vector<int> ids;
  std::vector<int64_t> steps;
  for (int i = 0; i < (int)c->slots.size(); ++i)
    if (c->slots[i].used) {
      ids.push_back(i);
      steps.push_back(n);
    }
  return step_many(c, ids, steps);
}

}  // namespace

// ---------------------------------------------------------------------------
// C ABI

extern "C" {

const char *lbm_strerror(int code) {
  switch (code) {
    case LBM_OK: return "ok";
    case LBM_EINVAL: return "invalid argument";
    case LBM_ENOMEM: return "out of memory or HBM budget";
    case LBM_EDEVICE: return "HIP runtime error";
    case LBM_EUNSTABLE: return "state is not finite";
    case LBM_ESTATE: return "wrong state";
    case LBM_ENOTSUP: return "not supported";
    default: return "unknown error";
  }
}

const char *lbm_last_error(void) { return g_last_error.c_str(); }

const char *lbm_version(void) { return "btrirt-lbm 0.1 gfx950"; }

int lbm_derive(const lbm_case *cs, lbm_lattice *out) {
  if (!out) return fail(LBM_EINVAL, "output is NULL");
  std::string why;
  int rc = derive(cs, out, why);
  if (rc != LBM_OK) return fail(rc, why);
  return LBM_OK;
}

size_t lbm_footprint(const lbm_case *cs) {
  lbm_lattice lat;
  std::string why;
  if (derive(cs, &lat, why) != LBM_OK) return 0;
  return layout_of(cs, lat).total;
}

int lbm_create(lbm_ctx **out, int device, void *hip_stream, size_t hbm_budget, int max_slots) {
  if (!out) return fail(LBM_EINVAL, "output is NULL");
  *out = nullptr;
  if (max_slots < 1 || max_slots > 1 << 16) return fail(LBM_EINVAL, "max_slots out of range");
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || ndev <= 0) {
    (void)hipGetLastError();
    return fail(LBM_EDEVICE, "no HIP device available");
  }
  if (device < 0 || device >= ndev) return fail(LBM_EINVAL, "device index out of range");
  HIP_TRY(hipSetDevice(device));
  lbm_ctx *c = new lbm_ctx();
  c->device = device;
  c->budget = hbm_budget;
  c->slots.resize(max_slots);
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, device) == hipSuccess && prop.multiProcessorCount > 0)
    c->num_cus = prop.multiProcessorCount;
  for (int prec = 0; prec < 2; ++prec)
    for (int steps = 2; steps <= 4; ++steps)
      for (int km = 0; km < lbm::kKernelModels; ++km)
        for (int staged = 0; staged < 2; ++staged)
          c->fused_wpc[prec][steps][km][staged] = lbm::fused_waves_per_cu(prec, steps, km, staged != 0);
  int rc = LBM_OK;
  if (hip_stream) {
    c->stream = static_cast<hipStream_t>(hip_stream);
  } else if (hipStreamCreate(&c->stream) != hipSuccess) {
    rc = fail(LBM_EDEVICE, "cannot create stream");
  } else {
    c->own_stream = true;
  }
  if (rc == LBM_OK &&
      (hipMalloc(&c->partials, (size_t)lbm::kRedBlocks * 16 * sizeof(double)) != hipSuccess ||
       hipMalloc(&c->stats_dev, sizeof(StatsDev)) != hipSuccess ||
       hipMalloc(&c->err_dev, sizeof(int32_t)) != hipSuccess ||
       hipHostMalloc(&c->err_host, sizeof(int32_t)) != hipSuccess ||
       hipHostMalloc(&c->stats_host, 2 * sizeof(StatsDev)) != hipSuccess))
    rc = fail(LBM_ENOMEM, "cannot allocate reduction scratch");
  if (rc == LBM_OK) {
    // the device is current: its copy of the static staging array
    const hipError_t e = hipGetSymbolAddress(&c->noalloc, HIP_SYMBOL(noalloc_scratch));
    if (e != hipSuccess || !c->noalloc) {
      c->noalloc = nullptr;
      rc = fail(LBM_EDEVICE, std::string("cannot resolve the static staging array: ") + hipGetErrorString(e));
    }
  }
  if (rc == LBM_OK) {
    *c->err_host = 0;
    if (lbm::launch_fill_zero(c->err_dev, sizeof(int32_t), c->stream) != hipSuccess ||
        hipStreamSynchronize(c->stream) != hipSuccess)
      rc = fail(LBM_EDEVICE, "cannot clear the device error word");
  }
  if (rc != LBM_OK) {
    lbm_destroy(c);
    return rc;
  }
  *out = c;
  return LBM_OK;
}

void lbm_destroy(lbm_ctx *c) {
  if (!c) return;
  (void)hipSetDevice(c->device);
  if (c->stream) (void)hipStreamSynchronize(c->stream);
  for (int i = 0; i < (int)c->slots.size(); ++i)
    if (c->slots[i].used) (void)lbm_release(c, i);
  free_batch(c);
  if (c->partials) (void)hipFree(c->partials);
  if (c->stats_dev) (void)hipFree(c->stats_dev);
  if (c->err_dev) (void)hipFree(c->err_dev);
  if (c->err_host) (void)hipHostFree(c->err_host);
  if (c->stats_host) (void)hipHostFree(c->stats_host);
  if (c->scratch) (void)hipFree(c->scratch);
  if (c->own_stream && c->stream) (void)hipStreamDestroy(c->stream);
  delete c;
}

int lbm_set_case(lbm_ctx *c, const lbm_case *cs, void *dev_buf, size_t buf_bytes,
                 int *slot_out) {
  TraceRange range("lbm_set_case");
  if (!c || !slot_out) return fail(LBM_EINVAL, "context or slot output is NULL");
  *slot_out = -1;
  lbm_lattice lat;
  std::string why;
  int rc = derive(cs, &lat, why);
  if (rc != LBM_OK) return fail(rc, why);
  int id = -1;
  for (int i = 0; i < (int)c->slots.size(); ++i)
    if (!c->slots[i].used) { id = i; break; }
  if (id < 0) return fail(LBM_ENOMEM, "no free slot");
  const Layout lay = layout_of(cs, lat);
  if (c->budget > 0 && c->used + lay.total > c->budget)
    return fail(LBM_ENOMEM, "case needs " + std::to_string(lay.total) + " bytes, " +
                                std::to_string(c->budget - c->used) + " left in the budget");
  HIP_TRY(hipSetDevice(c->device));
  void *base = nullptr;
  bool owned = false;
  if (dev_buf) {
    if (buf_bytes < lay.total)
      return fail(LBM_EINVAL, "lent buffer holds " + std::to_string(buf_bytes) + " bytes, " +
                                  std::to_string(lay.total) + " needed");
    if (reinterpret_cast<uintptr_t>(dev_buf) % kByteAlign != 0)
      return fail(LBM_EINVAL, "lent buffer must be 256-byte aligned");
    base = dev_buf;
  } else {
    if (hipMalloc(&base, lay.total) != hipSuccess) {
      (void)hipGetLastError();
      return fail(LBM_ENOMEM, "hipMalloc of " + std::to_string(lay.total) + " bytes failed");
    }
    owned = true;
  }
  Slot &s = c->slots[id];
  s = Slot();
  s.used = true;
  s.cs = *cs;
  s.lat = lat;
  s.lay = lay;
  s.base = base;
  s.owned = owned;
  s.dev = make_dev(cs, lat, lay, base);
  s.e0_dev = reinterpret_cast<StatsDev *>(static_cast<char *>(base) + lay.aux_off);
  c->used += lay.total;
  c->batch.dirty = true;
  hipError_t e = lbm::launch_init(s.dev, cs->precision, cs->init, cs->T0, cs->gauss_amp,
                                  cs->gauss_sigma, c->stream);
  if (e == hipSuccess && cs->pattern == LBM_PATTERN_AB)
    e = lbm::launch_fill_zero(s.dev.pop[1], lay.pop_bytes, c->stream);
  if (e != hipSuccess) {
    lbm_release(c, id);
    return fail(LBM_EDEVICE, std::string("init: ") + hipGetErrorString(e));
  }
  rc = restart_clock(c, s);
  if (rc != LBM_OK) {
    std::string msg = g_last_error;
    lbm_release(c, id);
    return fail(rc, msg);
  }
  *slot_out = id;
  return LBM_OK;
}

int lbm_release(lbm_ctx *c, int slot) {
  int rc = check_slot(c, slot);
  if (rc != LBM_OK) return rc;
  Slot &s = c->slots[slot];
  (void)hipStreamSynchronize(c->stream);
  drop_graphs(s);
  if (s.series) (void)hipFree(s.series);
  if (s.owned && s.base) (void)hipFree(s.base);
  c->used -= s.lay.total;
  s = Slot();
  c->batch.dirty = true;
  return LBM_OK;
}

int lbm_step(lbm_ctx *c, int slot, int64_t nsteps) {
  TraceRange range("lbm_step");
  if (!c) return fail(LBM_EINVAL, "context is NULL");
  if (nsteps < 0) return fail(LBM_EINVAL, "nsteps < 0");
  if (nsteps == 0) return LBM_OK;
  if (slot == LBM_ALL) return step_all(c, nsteps);
  int rc = check_slot(c, slot);
  if (rc != LBM_OK) return rc;
  return step_slot(c, c->slots[slot], nsteps);
}

int lbm_step_many(lbm_ctx *c, int count, const int32_t *slots, const int64_t *nsteps) {
  TraceRange range("lbm_step_many");
  if (!c) return fail(LBM_EINVAL, "context is NULL");
  if (count < 0 || (count > 0 && (!slots || !nsteps))) return fail(LBM_EINVAL, "bad slot list");
  std::vector<int> ids(count);
  std::vector<int64_t> n(count);
  for (int j = 0; j < count; ++j) {
    int rc = check_slot(c, slots[j]);
    if (rc != LBM_OK) return rc;
    if (nsteps[j] < 0) return fail(LBM_EINVAL, "negative step count");
    ids[j] = slots[j];
    n[j] = nsteps[j];
  }
  return step_many(c, ids, n);
}

int lbm_set_group_bytes(lbm_ctx *c, size_t bytes) {
  if (!c) return fail(LBM_EINVAL, "context is NULL");
  if (bytes < (size_t(1) << 20)) return fail(LBM_EINVAL, "group capacity below 1 MiB");
  c->group_bytes = bytes;
  c->batch.dirty = true;
  return LBM_OK;
}

int lbm_reduce(lbm_ctx *c, int slot, lbm_stats *out) {
  TraceRange range("lbm_reduce");
  int rc = check_slot(c, slot);
  if (rc != LBM_OK) return rc;
  if (!out) return fail(LBM_EINVAL, "output is NULL");
  Slot &s = c->slots[slot];
  StatsDev d{};
  double e0 = 0.0;
  rc = reduce_now(c, s, &d, &e0);
  if (rc != LBM_OK) return rc;
  fill_stats(s, d, e0, s.step, s.dev.parity, out);
  if (!out->finite) return fail(LBM_EUNSTABLE, "populations are not finite");
  return LBM_OK;
}

int lbm_fields(lbm_ctx *c, int slot, uint32_t mask, double *host, size_t n) {
  TraceRange range("lbm_fields");
  int rc = check_slot(c, slot);
  if (rc != LBM_OK) return rc;
  Slot &s = c->slots[slot];
  mask &= 63u;
  int planes = 0;
  for (int b = 0; b < 6; ++b) planes += (mask >> b) & 1u;
  const size_t cells = (size_t)s.cs.nx * s.cs.ny;
  if (!host || planes == 0 || n < planes * cells)
    return fail(LBM_EINVAL, "host buffer too small or empty mask");
  rc = ensure_scratch(c, planes * cells * sizeof(double));
  if (rc != LBM_OK) return rc;
  HIP_TRY(lbm::launch_fields(s.dev, s.cs.precision, mask, static_cast<double *>(c->scratch),
                             c->stream));
  HIP_TRY(hipMemcpyAsync(host, c->scratch, planes * cells * sizeof(double),
                         hipMemcpyDeviceToHost, c->stream));
  return sync_checked(c);
}

int lbm_fields_noalloc(lbm_ctx *c, int slot, uint32_t mask, double *host, size_t n) {
  TraceRange range("lbm_fields_noalloc");
  int rc = check_slot(c, slot);
  if (rc != LBM_OK) return rc;
  Slot &s = c->slots[slot];
  mask &= 63u;
  int planes = 0;
  for (int b = 0; b < 6; ++b) planes += (mask >> b) & 1u;
  const size_t cells = (size_t)s.cs.nx * s.cs.ny;
  if (!host || planes == 0 || n < planes * cells)
    return fail(LBM_EINVAL, "host buffer too small or empty mask");
  const size_t bytes = planes * cells * sizeof(double);
  if (bytes > kNoAllocBytes)
    return fail(LBM_EINVAL, "lbm_fields_noalloc: " + std::to_string(planes) + " field(s) of " +
                                std::to_string(cells) + " cells need " + std::to_string(bytes) +
                                " bytes of staging, above the fixed " + std::to_string(kNoAllocBytes) +
                                " bytes; ask for fewer fields or use lbm_fields");
  if (!c->noalloc) return fail(LBM_ESTATE, "static staging array not resolved for this device");
  HIP_TRY(lbm::launch_fields(s.dev, s.cs.precision, mask, static_cast<double *>(c->noalloc), c->stream));
  HIP_TRY(hipMemcpyAsync(host, c->noalloc, bytes, hipMemcpyDeviceToHost, c->stream));
  return sync_checked(c);
}

int lbm_set_report(lbm_ctx *c, int slot, int64_t every, int32_t capacity) {
  int rc = check_slot(c, slot);
  if (rc != LBM_OK) return rc;
  if (every < 0 || (every > 0 && capacity < 1)) return fail(LBM_EINVAL, "bad report schedule");
  Slot &s = c->slots[slot];
  HIP_TRY(hipStreamSynchronize(c->stream));
  if (s.series) (void)hipFree(s.series);
  s.series = nullptr;
  s.series_step.clear();
  s.series_parity.clear();
  s.report_every = every;
  s.report_cap = every > 0 ? capacity : 0;
  if (every > 0) {
    if (hipMalloc(&s.series, (size_t)capacity * sizeof(StatsDev)) != hipSuccess) {
      (void)hipGetLastError();
      s.series = nullptr;
      s.report_every = 0;
      s.report_cap = 0;
      return fail(LBM_ENOMEM, "cannot allocate the report ring");
    }
  }
  c->batch.dirty = true;
  return LBM_OK;
}

int lbm_series(lbm_ctx *c, int slot, lbm_stats *host, int32_t max, int32_t *count) {
  int rc = check_slot(c, slot);
  if (rc != LBM_OK) return rc;
  if (!count || (max > 0 && !host)) return fail(LBM_EINVAL, "bad output");
  Slot &s = c->slots[slot];
  const int32_t k = std::min<int32_t>((int32_t)s.series_step.size(), std::max<int32_t>(max, 0));
  *count = k;
  if (k == 0) return LBM_OK;
  std::vector<StatsDev> tmp(k);
  StatsDev e0{};
  rc = sync_checked(c);
  if (rc != LBM_OK) return rc;
  HIP_TRY(hipMemcpy(tmp.data(), s.series, k * sizeof(StatsDev), hipMemcpyDeviceToHost));
  HIP_TRY(hipMemcpy(&e0, s.e0_dev, sizeof(StatsDev), hipMemcpyDeviceToHost));
  for (int32_t j = 0; j < k; ++j)
    fill_stats(s, tmp[j], e0.total_H, s.series_step[j], s.series_parity[j], host + j);
  return LBM_OK;
}

int lbm_state_load(lbm_ctx *c, int slot, const double *f, const double *g, size_t n) {
  int rc = check_slot(c, slot);
  if (rc != LBM_OK) return rc;
  Slot &s = c->slots[slot];
  const size_t cnt = (size_t)lbm::kQ * s.cs.nx * s.cs.ny;
  if (!f || !g || n < cnt) return fail(LBM_EINVAL, "population buffers too small");
  rc = ensure_scratch(c, 2 * cnt * sizeof(double));
  if (rc != LBM_OK) return rc;
  double *df = static_cast<double *>(c->scratch);
  double *dg = df + cnt;
  HIP_TRY(hipMemcpyAsync(df, f, cnt * sizeof(double), hipMemcpyHostToDevice, c->stream));
  HIP_TRY(hipMemcpyAsync(dg, g, cnt * sizeof(double), hipMemcpyHostToDevice, c->stream));
  s.dev.parity = 0;
  HIP_TRY(lbm::launch_load(s.dev, s.cs.precision, df, dg, c->stream));
  drop_graphs(s);
  return restart_clock(c, s);
}

int lbm_state_save(lbm_ctx *c, int slot, double *f, double *g, size_t n) {
  int rc = check_slot(c, slot);
  if (rc != LBM_OK) return rc;
  Slot &s = c->slots[slot];
  const size_t cnt = (size_t)lbm::kQ * s.cs.nx * s.cs.ny;
  if (!f || !g || n < cnt) return fail(LBM_EINVAL, "population buffers too small");
  rc = ensure_scratch(c, 2 * cnt * sizeof(double));
  if (rc != LBM_OK) return rc;
  double *df = static_cast<double *>(c->scratch);
  double *dg = df + cnt;
  HIP_TRY(lbm::launch_save(s.dev, s.cs.precision, df, dg, c->stream));
  HIP_TRY(hipMemcpyAsync(f, df, cnt * sizeof(double), hipMemcpyDeviceToHost, c->stream));
  HIP_TRY(hipMemcpyAsync(g, dg, cnt * sizeof(double), hipMemcpyDeviceToHost, c->stream));
  return sync_checked(c);
}

int lbm_set_launch(lbm_ctx *c, int precision, int bx, int by, int cpl, int flags) {
  if (!c) return fail(LBM_EINVAL, "context is NULL");
  if (precision != LBM_FP64 && precision != LBM_FP32_SHIFTED) return fail(LBM_EINVAL, "precision");
  if (bx < 64 || bx % 64 != 0 || by < 1 || bx * by > 256 || (cpl != 1 && cpl != 2 && cpl != 4))
    return fail(LBM_EINVAL, "tile: bx multiple of 64, bx*by <= 256, cpl in {1,2,4}");
  LaunchCfg &L = c->launch[precision];
  L.bx = bx;
  L.by = by;
  L.cpl = cpl;
  L.xcd = (flags & LBM_LAUNCH_XCD_BANDS) ? 1 : 0;
  L.nt = (flags & LBM_LAUNCH_NONTEMPORAL) ? 1 : 0;
  L.reverse = (flags & LBM_LAUNCH_ALTERNATE) ? 1 : 0;
  L.zigzag = (flags & LBM_LAUNCH_ZIGZAG) ? 1 : 0;
  L.staged = (flags & LBM_LAUNCH_STAGED) ? 1 : 0;
  for (auto &s : c->slots) drop_graphs(s);
  drop_batch_graph(c);
  return LBM_OK;
}

int lbm_get_launch(lbm_ctx *c, int precision, int *bx, int *by, int *cpl, int *flags) {
  if (!c || !bx || !by || !cpl || !flags) return fail(LBM_EINVAL, "NULL argument");
  if (precision != LBM_FP64 && precision != LBM_FP32_SHIFTED) return fail(LBM_EINVAL, "precision");
  const LaunchCfg &L = c->launch[precision];
  *bx = L.bx;
  *by = L.by;
  *cpl = L.cpl;
  *flags = (L.xcd ? LBM_LAUNCH_XCD_BANDS : 0) | (L.nt ? LBM_LAUNCH_NONTEMPORAL : 0) |
           (L.reverse ? LBM_LAUNCH_ALTERNATE : 0) | (L.zigzag ? LBM_LAUNCH_ZIGZAG : 0) |
           (L.staged ? LBM_LAUNCH_STAGED : 0);
  return LBM_OK;
}

int lbm_set_fusion(lbm_ctx *c, int precision, int steps_per_launch, int segment_rows) {
  if (!c) return fail(LBM_EINVAL, "context is NULL");
  if (precision != LBM_FP64 && precision != LBM_FP32_SHIFTED) return fail(LBM_EINVAL, "precision");
  if (steps_per_launch < 1 || steps_per_launch > 4 || segment_rows < 0 ||
      segment_rows > lbm::kMaxSegmentRows)
    return fail(LBM_EINVAL, "steps per launch in {1, 2, 3, 4}, segment rows in 0..64");
  if (steps_per_launch == 4 && precision != LBM_FP32_SHIFTED)
    return fail(LBM_EINVAL, "four steps per launch are FP32 only");
  LaunchCfg &L = c->launch[precision];
  L.fuse = steps_per_launch;
  L.adapt = 0;
  if (segment_rows > 0)
    (steps_per_launch == 4 ? L.seg4 : (steps_per_launch == 3 ? L.seg3 : L.seg)) = segment_rows;
  for (auto &s : c->slots) drop_graphs(s);
  c->batch.dirty = true;  // item lists depend on the fusion
  drop_batch_graph(c);
  return LBM_OK;
}

int lbm_get_fusion(lbm_ctx *c, int precision, int *steps_per_launch, int *segment_rows) {
  if (!c || !steps_per_launch || !segment_rows) return fail(LBM_EINVAL, "NULL argument");
  if (precision != LBM_FP64 && precision != LBM_FP32_SHIFTED) return fail(LBM_EINVAL, "precision");
  const LaunchCfg &L = c->launch[precision];
  *steps_per_launch = L.fuse;
  *segment_rows = L.fuse == 4 ? L.seg4 : (L.fuse == 3 ? L.seg3 : L.seg);
  return LBM_OK;
}

int lbm_set_graph_chunk(lbm_ctx *c, int chunk) {
  if (!c) return fail(LBM_EINVAL, "context is NULL");
  if (chunk < 0 || chunk > 10000) return fail(LBM_EINVAL, "chunk out of range");
  HIP_TRY(hipStreamSynchronize(c->stream));
  c->graph_chunk = chunk;
  for (auto &s : c->slots) drop_graphs(s);
  drop_batch_graph(c);
  return LBM_OK;
}

int lbm_sync(lbm_ctx *c) {
  if (!c) return fail(LBM_EINVAL, "context is NULL");
  return sync_checked(c);
}

int lbm_stream(lbm_ctx *c, void **stream) {
  if (!c || !stream) return fail(LBM_EINVAL, "NULL argument");
  *stream = c->stream;
  return LBM_OK;
}

int lbm_slot_fusion(lbm_ctx *c, int slot, int *steps, int *rows) {
  int rc = check_slot(c, slot);
  if (rc != LBM_OK) return rc;
  if (!steps || !rows) return fail(LBM_EINVAL, "NULL argument");
  const Slot &s = c->slots[slot];
  const LaunchCfg L = slot_launch(c, s);
  *steps = steps_per_launch(c, s);
  *rows = *steps == 4 ? L.seg4 : (*steps == 3 ? L.seg3 : L.seg);
  return LBM_OK;
}

int lbm_slot_info(lbm_ctx *c, int slot, int64_t *step, int32_t *parity, size_t *bytes) {
  int rc = check_slot(c, slot);
  if (rc != LBM_OK) return rc;
  const Slot &s = c->slots[slot];
  if (step) *step = s.step;
  if (parity) *parity = s.dev.parity;
  if (bytes) *bytes = s.lay.total;
  return LBM_OK;
}

}  // extern "C"

// ---------------------------------------------------------------------------
// autotuner: times candidate tiles of the single-cavity step on a scratch
// cavity and keeps the fastest per (precision, size class)

namespace {

std::string size_class(int precision, int nx, int ny) {
  auto p2 = [](int v) { int p = 1; while (p < v) p <<= 1; return p; };
  return std::string(precision == LBM_FP64 ? "fp64" : "fp32s") + "/" + std::to_string(p2(nx)) +
         "x" + std::to_string(p2(ny));
}

// The cache is a flat JSON object {"<class>": [bx, by, cpl, flags, us_per_step], ...}.
std::map<std::string, std::vector<double>> read_cache(const char *path) {
  std::map<std::string, std::vector<double>> m;
  if (!path) return m;
  std::ifstream in(path);
  if (!in) return m;
  std::stringstream ss;
  ss << in.rdbuf();
  const std::string s = ss.str();
  size_t pos = 0;
  while ((pos = s.find('"', pos)) != std::string::npos) {
    const size_t end = s.find('"', pos + 1);
    if (end == std::string::npos) break;
    const std::string key = s.substr(pos + 1, end - pos - 1);
    const size_t lb = s.find('[', end), rb = s.find(']', end);
    if (lb == std::string::npos || rb == std::string::npos || rb < lb) break;
    std::vector<double> v;
    std::stringstream nums(s.substr(lb + 1, rb - lb - 1));
    std::string tok;
    while (std::getline(nums, tok, ',')) v.push_back(std::atof(tok.c_str()));
    if (v.size() >= 4) m[key] = v;
    pos = rb + 1;
  }
  return m;
}

void write_cache(const char *path, const std::map<std::string, std::vector<double>> &m) {
  if (!path) return;
  const std::string tmp = std::string(path) + ".tmp";
  std::ofstream out(tmp);
  if (!out) return;
  out << "{\n";
  size_t k = 0;
  for (const auto &kv : m) {
    out << "  \"" << kv.first << "\": [";
    for (size_t j = 0; j < kv.second.size(); ++j) out << (j ? ", " : "") << kv.second[j];
    out << "]" << (++k < m.size() ? "," : "") << "\n";
  }
  out << "}\n";
  out.close();
  std::rename(tmp.c_str(), path);
}

// Average ms of `reps` launches after two warm-up launches; each launch flips
// the scratch cavity's storage parity.
template <typename Launch>
int time_launches(lbm_ctx *c, CavDev &d, hipEvent_t e0, hipEvent_t e1, int reps, Launch launch,
                  float *ms) {
  hipError_t e = hipSuccess;
  for (int k = 0; k < 2 && e == hipSuccess; ++k) {
    e = launch(d);
    d.parity ^= 1;
  }
  e = e == hipSuccess ? hipEventRecord(e0, c->stream) : e;
  for (int k = 0; k < reps && e == hipSuccess; ++k) {
    e = launch(d);
    d.parity ^= 1;
  }
  e = e == hipSuccess ? hipEventRecord(e1, c->stream) : e;
  e = e == hipSuccess ? hipEventSynchronize(e1) : e;
  float t = 0.0f;
  e = e == hipSuccess ? hipEventElapsedTime(&t, e0, e1) : e;
  if (e != hipSuccess) return fail(LBM_EDEVICE, std::string("autotune: ") + hipGetErrorString(e));
  *ms = t / reps;
  return LBM_OK;
}

int flags_of(const LaunchCfg &L) {
  return (L.xcd ? LBM_LAUNCH_XCD_BANDS : 0) | (L.nt ? LBM_LAUNCH_NONTEMPORAL : 0) |
         (L.reverse ? LBM_LAUNCH_ALTERNATE : 0) | (L.zigzag ? LBM_LAUNCH_ZIGZAG : 0) |
         (L.staged ? LBM_LAUNCH_STAGED : 0);
}

}  // namespace

extern "C" int lbm_autotune(lbm_ctx *c, int precision, int nx, int ny, const char *cache_path) {
  if (!c) return fail(LBM_EINVAL, "context is NULL");
  if (precision != LBM_FP64 && precision != LBM_FP32_SHIFTED) return fail(LBM_EINVAL, "precision");
  const std::string key = size_class(precision, nx, ny);
  auto cache = read_cache(cache_path);
  auto it = cache.find(key);
  // the fastest depth per step among two, three and (FP32) four steps per
  // launch, unless the caller runs single steps
  auto pick = [&](int fuse, double us2, double us3, double us4) {
    if (fuse == 1) return 1;
    int f = us3 / 3 < us2 / 2 ? 3 : 2;
    if (precision == LBM_FP32_SHIFTED && us4 / 4 < (f == 3 ? us3 / 3 : us2 / 2)) f = 4;
    return f;
  };
  // entries without the three-step timing, or FP32 entries without the
  // four-step timing (older formats), are tuned again
  const size_t need = precision == LBM_FP32_SHIFTED ? 11 : 9;
  if (it != cache.end() && it->second.size() >= need) {
    const std::vector<double> &v = it->second;
    const int fuse = c->launch[precision].fuse;
    int rc = lbm_set_launch(c, precision, (int)v[0], (int)v[1], (int)v[2], (int)v[3]);
    if (rc == LBM_OK) {
      rc = lbm_set_fusion(c, precision, 2, (int)v[5]);
      if (rc == LBM_OK) rc = lbm_set_fusion(c, precision, 3, (int)v[7]);
      if (rc == LBM_OK && need == 11) rc = lbm_set_fusion(c, precision, 4, (int)v[9]);
      if (rc == LBM_OK)
        rc = lbm_set_fusion(c, precision, pick(fuse, v[6], v[8], need == 11 ? v[10] : 1e30), 0);
    }
    return rc;
  }
  // scratch cavity on two lattices: the one-step candidates run in place on
  // its first lattice, the two-step candidates on both
  lbm_case cs{};
  cs.nx = nx;
  cs.ny = ny;
  cs.precision = precision;
  cs.pattern = LBM_PATTERN_AB;
  cs.param_mode = LBM_PARAM_DIMENSIONLESS;
  cs.init = LBM_INIT_SOLID_AT_TM;
  cs.Ra = 1e6; cs.Pr = 1.0; cs.Ste = 1.0; cs.Ma = 0.1;
  cs.Cp = 1.0; cs.Th = 1.0; cs.Tm = 0.0; cs.rho0 = 1.0;
  cs.heater_center = 0.5; cs.heater_width = 0.25;
  cs.k0_g = cs.k2_g = cs.k0_f = cs.k1_f = std::nan("");
  cs.gauss_sigma = 1.0;
  cs.darcy_c = cs.darcy_eps = std::nan("");
  lbm_lattice lat;
  std::string why;
  if (derive(&cs, &lat, why) != LBM_OK) return fail(LBM_EINVAL, why);
  const Layout lay = layout_of(&cs, lat);
  void *base = nullptr;
  if (hipMalloc(&base, lay.total) != hipSuccess) {
    (void)hipGetLastError();
    return fail(LBM_ENOMEM, "autotune scratch cavity does not fit");
  }
  CavDev two = make_dev(&cs, lat, lay, base);
  CavDev one = two;
  one.pattern = LBM_PATTERN_AA;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  int rc = LBM_OK;
  const LaunchCfg saved = c->launch[precision];
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess ||
      lbm::launch_init(two, precision, LBM_INIT_SOLID_AT_TM, 0, 0, 1, c->stream) != hipSuccess ||
      lbm::launch_fill_zero(two.cumq, lay.cumq_bytes, c->stream) != hipSuccess) {
    rc = fail(LBM_EDEVICE, "autotune set-up failed");
  }
  const int reps = 10;
  // one step per launch: block shape, rows per lane, walk flags
  LaunchCfg best = saved;
  float best_ms = 1e30f;
  const int shapes[][2] = {{64, 1}, {64, 2}, {64, 4}, {128, 1}, {128, 2}, {256, 1}};
  const int cpls[] = {1, 2, 4};
  for (const auto &sh : shapes) {
    for (int cpl : cpls) {
      for (int flags = 0; flags < 8 && rc == LBM_OK; ++flags) {
        LaunchCfg cfg = saved;
        cfg.bx = sh[0];
        cfg.by = sh[1];
        cfg.cpl = cpl;
        cfg.xcd = flags & LBM_LAUNCH_XCD_BANDS ? 1 : 0;
        cfg.nt = flags & LBM_LAUNCH_NONTEMPORAL ? 1 : 0;
        cfg.reverse = flags & LBM_LAUNCH_ALTERNATE ? 1 : 0;
        float ms = 0.0f;
        rc = time_launches(c, one, e0, e1, reps,
                           [&](const CavDev &d) { return lbm::launch_step(d, precision, cfg, c->stream); },
                           &ms);
        if (rc == LBM_OK && ms < best_ms) {
          best_ms = ms;
          best = cfg;
        }
      }
    }
  }
  // two steps per launch: segment rows, rows staged or loaded directly
  int best_seg = saved.seg, best_staged = saved.staged;
  float best2_ms = 1e30f;
  const int segs[] = {1, 2, 3, 4, 6, 8};
  for (int seg : segs) {
    for (int staged = 0; staged < 2 && rc == LBM_OK; ++staged) {
      LaunchCfg cfg = best;
      cfg.zigzag = 1;
      cfg.seg = seg;
      cfg.staged = staged;
      float ms = 0.0f;
      rc = time_launches(c, two, e0, e1, reps,
                         [&](const CavDev &d) { return lbm::launch_step2(d, precision, cfg, c->stream); },
                         &ms);
      if (rc == LBM_OK && ms < best2_ms) {
        best2_ms = ms;
        best_seg = seg;
        best_staged = staged;
      }
    }
  }
  // three steps per launch: segment rows (rows always staged)
  int best_seg3 = saved.seg3;
  float best3_ms = 1e30f;
  const int segs3[] = {2, 4, 6, 8, 12};
  for (int seg : segs3) {
    if (rc != LBM_OK) break;
    LaunchCfg cfg = best;
    cfg.zigzag = 1;
    cfg.seg3 = seg;
    float ms = 0.0f;
    rc = time_launches(c, two, e0, e1, reps,
                       [&](const CavDev &d) { return lbm::launch_step3(d, precision, cfg, c->stream); },
                       &ms);
    if (rc == LBM_OK && ms < best3_ms) {
      best3_ms = ms;
      best_seg3 = seg;
    }
  }
  // four steps per launch (FP32): segment rows (rows always staged)
  int best_seg4 = saved.seg4;
  float best4_ms = 1e30f;
  if (precision == LBM_FP32_SHIFTED) {
    for (int seg : segs3) {
      if (rc != LBM_OK) break;
      LaunchCfg cfg = best;
      cfg.zigzag = 1;
      cfg.seg4 = seg;
      float ms = 0.0f;
      rc = time_launches(c, two, e0, e1, reps,
                         [&](const CavDev &d) { return lbm::launch_step4(d, precision, cfg, c->stream); },
                         &ms);
      if (rc == LBM_OK && ms < best4_ms) {
        best4_ms = ms;
        best_seg4 = seg;
      }
    }
  }
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  (void)hipStreamSynchronize(c->stream);
  (void)hipFree(base);
  if (rc != LBM_OK) {
    c->launch[precision] = saved;
    return rc;
  }
  best.zigzag = 1;
  best.staged = best_staged;
  const int best_flags = flags_of(best);
  // entry: bx, by, cpl, flags, us per one-step launch, segment rows and us
  // per launch of the two-step kernel, the same of the three-step kernel and
  // (FP32) of the four-step kernel
  cache[key] = {(double)best.bx, (double)best.by, (double)best.cpl, (double)best_flags,
                1000.0 * best_ms, (double)best_seg, 1000.0 * best2_ms, (double)best_seg3,
                1000.0 * best3_ms};
  if (precision == LBM_FP32_SHIFTED) {
    cache[key].push_back((double)best_seg4);
    cache[key].push_back(1000.0 * best4_ms);
  }
  write_cache(cache_path, cache);
  rc = lbm_set_launch(c, precision, best.bx, best.by, best.cpl, best_flags);
  if (rc == LBM_OK) rc = lbm_set_fusion(c, precision, 2, best_seg);
  if (rc == LBM_OK) rc = lbm_set_fusion(c, precision, 3, best_seg3);
  if (rc == LBM_OK && precision == LBM_FP32_SHIFTED) rc = lbm_set_fusion(c, precision, 4, best_seg4);
  if (rc == LBM_OK)
    rc = lbm_set_fusion(c, precision,
                        pick(saved.fuse, 1000.0 * best2_ms, 1000.0 * best3_ms, 1000.0 * best4_ms), 0);
  return rc;
}

// ---------------------------------------------------------------------------
// checkpoints: the slot's device region as stored, behind a small header

namespace {

struct CheckpointHeader {
  char magic[8];
  uint32_t version, header_bytes;
  int32_t precision, pattern, parity, pad;
  int64_t step;
  uint64_t region_bytes;
  lbm_case cs;
};

constexpr char kMagic[8] = {'B', 'T', 'R', 'I', 'R', 'T', 'C', 'K'};

}  // namespace

extern "C" int lbm_stream_probe(lbm_ctx *c, size_t bytes, int pattern, int launches, double *us) {
  TraceRange range("lbm_stream_probe");
  if (!c || !us) return fail(LBM_EINVAL, "NULL argument");
  if (pattern != LBM_PATTERN_AA && pattern != LBM_PATTERN_AB) return fail(LBM_EINVAL, "pattern");
  if (launches < 1 || launches > 100000) return fail(LBM_EINVAL, "launches out of range (1 .. 100000)");
  const size_t chunk = (size_t)lbm::kPlanes * lbm::kWave * sizeof(double);
  const int64_t chunks = (int64_t)(bytes / chunk);
  if (chunks < 1 || chunks > ((int64_t)INT32_MAX - 3)) return fail(LBM_EINVAL, "bytes out of range");
  HIP_TRY(hipSetDevice(c->device));
  HIP_TRY(hipStreamSynchronize(c->stream));
  const size_t n = (size_t)chunks * chunk;
  void *a = nullptr, *b = nullptr;
  if (hipMalloc(&a, n) != hipSuccess ||
      (pattern == LBM_PATTERN_AB && hipMalloc(&b, n) != hipSuccess)) {
    (void)hipGetLastError();
    if (a) (void)hipFree(a);
    return fail(LBM_ENOMEM, "stream probe buffers do not fit");
  }
  if (!b) b = a;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  int rc = LBM_OK;
  float ms = 0.0f;
  auto launch = [&](int i) {
    // two lattices: odd launches copy back; both patterns walk backwards on odd launches
    const bool odd = (i & 1) != 0;
    const double *src = static_cast<const double *>(odd ? b : a);
    double *dst = static_cast<double *>(odd ? a : b);
    return lbm::launch_stream(src, dst, chunks, odd, c->stream);
  };
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess ||
      lbm::launch_fill_zero(a, n, c->stream) != hipSuccess ||
      (b != a && lbm::launch_fill_zero(b, n, c->stream) != hipSuccess) || launch(0) != hipSuccess ||
      launch(1) != hipSuccess || hipEventRecord(e0, c->stream) != hipSuccess) {
    rc = fail(LBM_EDEVICE, "stream probe set-up failed");
  }
  for (int i = 0; rc == LBM_OK && i < launches; ++i)
    if (launch(i) != hipSuccess) rc = fail(LBM_EDEVICE, "stream probe launch failed");
  if (rc == LBM_OK && (hipEventRecord(e1, c->stream) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
                       hipEventElapsedTime(&ms, e0, e1) != hipSuccess))
    rc = fail(LBM_EDEVICE, "stream probe timing failed");
  (void)hipStreamSynchronize(c->stream);
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  if (b != a) (void)hipFree(b);
  (void)hipFree(a);
  if (rc == LBM_OK) *us = 1e3 * (double)ms / launches;
  return rc;
}

extern "C" size_t lbm_checkpoint_bytes(lbm_ctx *c, int slot) {
  if (check_slot(c, slot) != LBM_OK) return 0;
  return sizeof(CheckpointHeader) + c->slots[slot].lay.total;
}

extern "C" int lbm_checkpoint_save(lbm_ctx *c, int slot, void *host, size_t n) {
  int rc = check_slot(c, slot);
  if (rc != LBM_OK) return rc;
  Slot &s = c->slots[slot];
  const size_t need = sizeof(CheckpointHeader) + s.lay.total;
  if (!host || n < need) return fail(LBM_EINVAL, "checkpoint buffer holds fewer than " + std::to_string(need) + " bytes");
  CheckpointHeader h{};
  std::memcpy(h.magic, kMagic, sizeof(kMagic));
  h.version = 1;
  h.header_bytes = sizeof(CheckpointHeader);
  h.precision = s.cs.precision;
  h.pattern = s.cs.pattern;
  h.parity = s.dev.parity;
  h.step = s.step;
  h.region_bytes = s.lay.total;
  h.cs = s.cs;
  std::memcpy(host, &h, sizeof(h));
  HIP_TRY(hipMemcpyAsync(static_cast<char *>(host) + sizeof(h), s.base, s.lay.total,
                         hipMemcpyDeviceToHost, c->stream));
  HIP_TRY(hipStreamSynchronize(c->stream));
  return LBM_OK;
}

namespace {

// Checks a checkpoint on the host without touching any device: header, the
// embedded case (derived as lbm_set_case would), and the agreement of the
// header's precision, pattern and region size with that case.
int validate_checkpoint(const void *host, size_t n, CheckpointHeader *h, lbm_lattice *lat,
                        Layout *lay) {
  if (!host || n < sizeof(*h)) return fail(LBM_EINVAL, "checkpoint too short");
  std::memcpy(h, host, sizeof(*h));
  if (std::memcmp(h->magic, kMagic, sizeof(kMagic)) != 0 || h->version != 1 ||
      h->header_bytes != sizeof(*h))
    return fail(LBM_EINVAL, "not a checkpoint of this library version");
  if (h->parity != 0 && h->parity != 1) return fail(LBM_EINVAL, "corrupt checkpoint parity");
  if (h->step < 0) return fail(LBM_EINVAL, "corrupt checkpoint step counter");
  std::string why;
  if (derive(&h->cs, lat, why) != LBM_OK) return fail(LBM_EINVAL, "checkpoint case invalid: " + why);
  if (h->cs.precision != h->precision || h->cs.pattern != h->pattern)
    return fail(LBM_EINVAL, "checkpoint header and its case disagree on precision or pattern");
  *lay = layout_of(&h->cs, *lat);
  if (lay->total != h->region_bytes)
    return fail(LBM_EINVAL, "checkpoint region of " + std::to_string(h->region_bytes) +
                                " bytes does not match its case (" + std::to_string(lay->total) + ")");
  if (n - sizeof(*h) < h->region_bytes) return fail(LBM_EINVAL, "checkpoint truncated");
  return LBM_OK;
}

}  // namespace

extern "C" int lbm_checkpoint_info(const void *host, size_t n, lbm_case *cs, int64_t *step) {
  CheckpointHeader h{};
  lbm_lattice lat;
  Layout lay;
  const int rc = validate_checkpoint(host, n, &h, &lat, &lay);
  if (rc != LBM_OK) return rc;
  if (cs) *cs = h.cs;
  if (step) *step = h.step;
  return LBM_OK;
}

extern "C" int lbm_checkpoint_load(lbm_ctx *c, int slot, const void *host, size_t n) {
  int rc = check_slot(c, slot);
  if (rc != LBM_OK) return rc;
  Slot &s = c->slots[slot];
  CheckpointHeader h{};
  lbm_lattice lat;
  Layout lay;
  rc = validate_checkpoint(host, n, &h, &lat, &lay);
  if (rc != LBM_OK) return rc;
  if (h.cs.nx != s.cs.nx || h.cs.ny != s.cs.ny || h.cs.precision != s.cs.precision ||
      h.cs.pattern != s.cs.pattern || lay.total != s.lay.total)
    return fail(LBM_EINVAL, "checkpoint was taken from a cavity of another size, precision or pattern");
  // everything is checked: only now does the slot change
  rc = sync_checked(c);
  if (rc != LBM_OK) return rc;
  HIP_TRY(hipMemcpyAsync(s.base, static_cast<const char *>(host) + sizeof(h), s.lay.total,
                         hipMemcpyHostToDevice, c->stream));
  HIP_TRY(hipStreamSynchronize(c->stream));
  // the physics of the restored run is the checkpoint's
  s.cs = h.cs;
  s.lat = lat;
  s.dev = make_dev(&s.cs, s.lat, s.lay, s.base);
  s.dev.parity = h.parity;
  s.step = h.step;
  s.series_step.clear();
  s.series_parity.clear();
  drop_graphs(s);
  c->batch.dirty = true;
  return LBM_OK;
}
