// Internal interface between the host runtime and the gfx950 kernels.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <string>

namespace lbm {

constexpr int kQ = 9;
constexpr int kPlanes = 2 * kQ;  // f_0..f_8 then g_0..g_8
constexpr int kWave = 64;
constexpr int kXcds = 8;
// How the solid holds the flow still (values of LBM_SOLID_* in lbm.h).
constexpr int kSolidScale = 0, kSolidDarcy = 1, kSolidPbb = 2;
// Kernel variants of the fused and batched kernels: the three solid models,
// and the scaled-velocity model with k0 = 1 for both populations, where the
// (1 - k0) p term of Eq. (2) vanishes, so the collision skips it and the
// pre-collision populations are dead once their moments are taken.  Its
// results equal the general collision's with those rates (a multiply by an
// exact zero dropped; only the sign of a zero sum can differ).
constexpr int kScaleUnitK0 = 3;
constexpr int kKernelModels = 4;

// The rates of Eq. (2) and the constants of one cavity in the combinations
// that the collision multiplies by (its pair form, lbm_device.h), in the
// arithmetic type R of the update.  Computed once on the host, so that no
// kernel spends instructions on them; kernels read them from the cavity
// descriptor into scalar registers.
template <typename R>
struct Rates {
  R omk0g, omk0f;          // 1 - k0 for g and f
  R k0g, k0g9;             // k0 and k0/9 for g
  R dk1g3, k1g3, dk2g6;    // (k1 - k0)/3, k1/3, (k2 - k0)/6 for g
  R k0f9, k0h, k0e;        // k0/9, k0/2, k0/8 for f
  R dk1f3, k1f3, dk2f6;    // (k1 - k0)/3, k1/3, (k2 - k0)/6 for f
  R hk1f3, hk2f3;          // (1 - k1/2)/3, (1 - k2/2)/3: force terms of f
  R CpTm, L, inv_L, inv_Cp, rho0, inv_rho0;
  R gbc;                   // rho0 g beta / Cp: buoyancy per unit of Cp theta
  R c2[3];                 // 2 w_i Cp (Th - Tm) for w = 4/9, 1/9, 1/36
  R darcy_c, darcy_eps;    // drag constants of the Darcy solid model

  __host__ __device__ R anti(int i) const { return i == 0 ? c2[0] : (i <= 4 ? c2[1] : c2[2]); }
};

// Everything a kernel needs to advance or inspect one cavity.  Built on the
// host from a validated case; passed by value (single cavity) or read from a
// device array (batched launch).
struct CavDev {
  int32_t nx, ny, pitch;
  int32_t periodic_x, periodic_y;
  int32_t hlo, hhi;    // heated cells [hlo, hhi] of row 0; none when hlo > hhi
  int32_t parity;      // in-place pattern: 0 natural, 1 swapped; AB: index of current lattice
  int32_t pattern;     // 0 in place (A-A), 1 two lattices
  int32_t active_steps; // batched launch: launches of the current chunk that advance it
  int32_t solid_model;  // LBM_SOLID_*
  int32_t kmodel;       // kernel variant: solid_model, or kScaleUnitK0 (set_rates)
  int64_t plane;       // elements between consecutive population planes of a cell
  // relaxation rates of Eq. (2)
  double k0g, k1g, k2g, k0f, k1f, k2f;
  double Cp, inv_Cp, latent, inv_latent, rho0, inv_rho0;
  double gbeta_rho0;   // rho0 * g * beta
  double dT;           // Th - Tm
  double Tm;
  double alpha;
  double darcy_c, darcy_eps;  // LBM_SOLID_DARCY: A = C (1 - fl)^2 / (fl^3 + eps)
  void *pop[2];        // population planes (pop[1] only for two lattices)
  double *cumq;        // per-column strip enthalpy summed over steps, nx doubles
  Rates<double> r64;   // the rates for each arithmetic type (set_rates)
  Rates<float> r32;
};

template <typename R>
inline Rates<R> make_rates(const CavDev &c) {
  Rates<R> k;
  k.omk0g = R(1.0 - c.k0g);
  k.omk0f = R(1.0 - c.k0f);
  k.k0g = R(c.k0g);
  k.k0g9 = R(c.k0g / 9.0);
  k.dk1g3 = R((c.k1g - c.k0g) / 3.0);
  k.k1g3 = R(c.k1g / 3.0);
  k.dk2g6 = R((c.k2g - c.k0g) / 6.0);
  k.k0f9 = R(c.k0f / 9.0);
  k.k0h = R(c.k0f / 2.0);
  k.k0e = R(c.k0f / 8.0);
  k.dk1f3 = R((c.k1f - c.k0f) / 3.0);
  k.k1f3 = R(c.k1f / 3.0);
  k.dk2f6 = R((c.k2f - c.k0f) / 6.0);
  k.hk1f3 = R((1.0 - 0.5 * c.k1f) / 3.0);
  k.hk2f3 = R((1.0 - 0.5 * c.k2f) / 3.0);
  k.CpTm = R(c.Cp * c.Tm);
  k.L = R(c.latent);
  k.inv_L = R(c.inv_latent);
  k.inv_Cp = R(c.inv_Cp);
  k.rho0 = R(c.rho0);
  k.inv_rho0 = R(c.inv_rho0);
  k.gbc = R(c.gbeta_rho0 * c.inv_Cp);
  k.c2[0] = R(2.0 * (4.0 / 9.0) * c.Cp * c.dT);
  k.c2[1] = R(2.0 * (1.0 / 9.0) * c.Cp * c.dT);
  k.c2[2] = R(2.0 * (1.0 / 36.0) * c.Cp * c.dT);
  k.darcy_c = R(c.darcy_c);
  k.darcy_eps = R(c.darcy_eps);
  return k;
}

// Fills the rate tables and the kernel variant of a descriptor whose other
// fields are set.
inline void set_rates(CavDev &c) {
  c.r64 = make_rates<double>(c);
  c.r32 = make_rates<float>(c);
  const bool unit_k0 = c.k0g == 1.0 && c.k0f == 1.0 && c.r64.omk0g == 0.0 && c.r64.omk0f == 0.0 &&
                       c.r32.omk0g == 0.0f && c.r32.omk0f == 0.0f;
  c.kmodel = c.solid_model == kSolidScale && unit_k0 ? kScaleUnitK0 : c.solid_model;
}

// Batched launch: tiles of many cavities in one grid.
struct BatchTile {
  int32_t cav;   // index into the CavDev array
  int32_t x0, y0;
  int32_t pad;
};

struct LaunchCfg {
  int bx = 256, by = 1, cpl = 1;
  int xcd = 1;  // contiguous tile bands per XCD
  int nt = 0;   // non-temporal population loads and stores
  int reverse = 1;  // walk tiles backwards on odd storage parity
  int zigzag = 1;   // two-step kernel: odd segments walked downwards
  int staged = 1;   // two-step kernel: rows copied into LDS one row ahead
  int fuse = 2;     // steps per launch of the two-lattice pattern (1, 2, 3, or 4 in FP32)
  int seg = 4;      // rows per wavefront segment of the two-step kernel
  int seg3 = 6;     // rows per wavefront segment of the three-step kernel
  int seg4 = 6;     // rows per wavefront segment of the four-step kernel (FP32)
  int adapt = 1;    // default fusion: depth and three-step segments follow the cavity size
};
constexpr int kMaxSegmentRows = 64;
constexpr int kStripCols = kWave - 2;   // owned columns of a two-step wavefront
constexpr int kStrip3Cols = kWave - 4;  // owned columns of a three-step wavefront
constexpr int kStrip4Cols = kWave - 6;  // owned columns of a four-step wavefront

// Defaults per precision, the fastest measured on MI355X at 2048x1024 and
// 4096x2048: three steps per launch in segments of 4 rows (FP64) or 6 rows
// (FP32), four-step segments of 6 rows; two-step launches (the batched path,
// shorter remainders) in segments of 2 rows (FP64) or 4 rows (FP32).
inline LaunchCfg default_launch(int precision) {
  LaunchCfg L;
  L.fuse = 3;
  L.seg = precision == 0 ? 2 : 4;
  L.seg3 = precision == 0 ? 4 : 6;
  return L;
}

// Accumulators of one reduction, FP64.
enum RedSlot {
  kRedFl = 0, kRedH, kRedRho, kRedQ, kRedFields  // compensated sums
};

// Diagnostics on the device (same order as lbm_stats minus host-only fields).
struct StatsDev {
  double melt_fraction, heater_q, total_H, heat_in_cum, mass, max_u;
  double nonfinite;
  double pad;
};

// Device error word of a context: set by a batched kernel whose work-list
// header is empty or out of range (a host bookkeeping fault); the launch then
// advances nothing.
constexpr int32_t kErrBatchHeader = 1;

// The header {first, count} of a batched launch addresses items [first,
// first + count) of a list of cap entries.
__device__ __forceinline__ bool batch_header_ok(int first, int count, int cap) {
  return first >= 0 && count > 0 && first <= cap - count;
}

constexpr int kRedBlocks = 512;   // fixed grid of the reduction (deterministic order)
constexpr int kRedThreads = 256;

// Launchers (all asynchronous on `s`); return hipSuccess or the launch error.
hipError_t launch_init(const CavDev &c, int precision, int mode, double T0, double amp,
                       double sigma, hipStream_t s);
hipError_t launch_step(const CavDev &c, int precision, const LaunchCfg &cfg, hipStream_t s);
// Two steps of the two-lattice pattern in one launch: reads pop[parity],
// writes pop[parity ^ 1].
hipError_t launch_step2(const CavDev &c, int precision, const LaunchCfg &cfg, hipStream_t s);
// Three steps per launch (two-lattice pattern): FP32 stages rows through LDS,
// FP64 keeps its level-2 window there and loads rows directly.
hipError_t launch_step3(const CavDev &c, int precision, const LaunchCfg &cfg, hipStream_t s);
// four steps per launch, FP32 only (hipErrorInvalidValue for FP64)
hipError_t launch_step4(const CavDev &c, int precision, const LaunchCfg &cfg, hipStream_t s);
// hdr_dev: {first tile, tile count} of this launch; tiles_dev holds tile_cap
// entries.  A header that is empty or points outside them advances nothing
// and sets *err_dev to kErrBatchHeader, which the host reports as an error.
// model: the kernel variant shared by every cavity of the list (CavDev::kmodel).
hipError_t launch_step_batch(const CavDev *cavs_dev, const BatchTile *tiles_dev,
                             const int32_t *hdr_dev, int tile_cap, int precision, int model,
                             int tile_bx, int tile_rows, int launch_index, int grid,
                             int32_t *err_dev, hipStream_t s);
// Batched two-step launch over wavefront items {cavity, strip origin x0,
// segment origin y0, segment index} of two-lattice cavities: launch j
// advances cavity c by two steps while 2 j + 2 <= active_steps(c), by one
// step when 2 j + 1 == active_steps(c), else leaves it.
hipError_t launch_step2_batch(const CavDev *cavs_dev, const BatchTile *items_dev,
                              const int32_t *hdr_dev, int item_cap, int precision, int model,
                              const LaunchCfg &cfg, int launch_index, int grid, int32_t *err_dev,
                              hipStream_t s);
// Batched three-step launch over 60-column strip segments (cfg.seg3 rows):
// launch j advances cavity c by three steps while 3 j + 3 <= active_steps(c),
// by the one or two steps left when 3 j < active_steps(c) < 3 j + 3, else
// leaves it.
hipError_t launch_step3_batch(const CavDev *cavs_dev, const BatchTile *items_dev,
                              const int32_t *hdr_dev, int item_cap, int precision, int model,
                              const LaunchCfg &cfg, int launch_index, int grid, int32_t *err_dev,
                              hipStream_t s);
// Workgroups of a batched two- or three-step launch that fill the device once.
int step2_batch_grid(int num_cus);
// Wavefronts of a single-cavity launch fusing `steps` (2, 3 or 4) steps that
// one CU holds at once, from the occupancy of the kernel instance for that
// precision, kernel variant and (two steps) row staging; 0 if unknown.
int fused_waves_per_cu(int precision, int steps, int kmodel, bool staged);
hipError_t launch_reduce(const CavDev &c, int precision, double *partials, StatsDev *out,
                         hipStream_t s);
hipError_t launch_fields(const CavDev &c, int precision, uint32_t mask, double *out,
                         hipStream_t s);
hipError_t launch_load(const CavDev &c, int precision, const double *f, const double *g,
                       hipStream_t s);
hipError_t launch_save(const CavDev &c, int precision, double *f, double *g, hipStream_t s);
hipError_t launch_fill_zero(void *p, size_t bytes, hipStream_t s);
// chunks of 18 x 64 doubles from src to dst (dst == src: in place); back: walk order reversed
hipError_t launch_stream(const double *src, double *dst, int64_t chunks, int back, hipStream_t s);
hipError_t launch_copy_stats(const StatsDev *src, StatsDev *dst, hipStream_t s);

// Records the message returned by lbm_last_error() on this thread.
void set_last_error(const std::string &msg);

}  // namespace lbm
