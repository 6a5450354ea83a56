// Two time steps per launch for the two-lattice pattern (temporal blocking).
//
// One launch reads the natural state at time t from lattice A once and writes
// the natural state at t+2 to lattice B once, so a pair of steps moves the
// bytes of one.  Each wavefront owns a strip of 62 columns and a segment of
// SEG rows and walks up the segment with a three-row window in registers:
//   - first step ("P1", a collision of the loaded state) for rows y0-1 .. y1,
//     columns x0-1 .. x0+62 (one halo column/row on each side, recomputed by
//     the neighbouring wavefronts as well);
//   - second step for the owned cells: the streamed populations are taken
//     from the window (from the neighbouring lane for x shifts, a wavefront
//     shuffle), walls reflect into the cell's own first-step values exactly as
//     the single-step kernels do, the collision runs again and the result is
//     scattered to B.
// Only registers and lane shuffles hold the intermediate state; nothing is
// staged in memory between the two steps.  Every collision is the same code
// as in the single-step kernels, so a launch equals two single two-lattice
// steps bit for bit.
#include "lbm_device.h"

namespace lbm {
namespace {

using namespace dev;

constexpr int kStripCols = kWave - 2;  // owned columns per wavefront

// Populations going up (c_y = +1): 2, 5, 6 -> slots 0, 1, 2 of the window.
__device__ constexpr int up_slot(int i) { return i == 2 ? 0 : (i == 5 ? 1 : 2); }

template <typename R>
__device__ __forceinline__ R lane_from(R v, int dx) {
  // value of the lane holding column x - dx
  if (dx > 0) return __shfl_up(v, 1, kWave);
  if (dx < 0) return __shfl_down(v, 1, kWave);
  return v;
}

template <typename S, typename R, int SEG>
__global__ __launch_bounds__(256) void k_step2(CavDev c, int strips_x, int nseg, int order) {
  const int lane = threadIdx.x & (kWave - 1);
  const int b = tile_of(blockIdx.x, gridDim.x, order & 1, (order & 2) && (c.parity & 1));
  const int w = b * (blockDim.x / kWave) + (threadIdx.x / kWave);
  if (w >= strips_x * nseg) return;  // uniform per wavefront; no barriers follow
  const int strip = w % strips_x, seg = w / strips_x;
  const int x = strip * kStripCols - 1 + lane;
  const int y0 = seg * SEG;
  const int y1 = min(y0 + SEG, c.ny);
  // only columns -1 .. nx matter (owners are 0 .. nx-1); with periodic sides
  // the halo columns -1 and nx wrap once
  const bool x_real = (x >= 0 && x < c.nx) || (c.periodic_x && (x == -1 || x == c.nx));
  const int xw = x < 0 ? x + c.nx : (x >= c.nx ? x - c.nx : x);
  const bool owner = lane >= 1 && lane <= kStripCols && x < c.nx;
  const bool bottom_hot = !c.periodic_y && x >= c.hlo && x <= c.hhi;
  const Coef<R> k(c);
  const S *__restrict__ A = static_cast<const S *>(c.parity ? c.pop[1] : c.pop[0]);
  S *__restrict__ B = static_cast<S *>(c.parity ? c.pop[0] : c.pop[1]);

  // first step of row r: the loaded natural state collided (zeros when the
  // row or column does not exist; such values are never used)
  auto first_step = [&](int r, R (&f)[kQ], R (&g)[kQ]) {
    const bool r_real = (r >= 0 && r < c.ny) || (c.periodic_y && (r == -1 || r == c.ny));
    if (!(r_real && x_real)) {
#pragma unroll
      for (int i = 0; i < kQ; ++i) f[i] = g[i] = R(0);
      return;
    }
    const int rw = r < 0 ? r + c.ny : (r >= c.ny ? r - c.ny : r);
    load_natural<S, R>(A, c.plane, cell_base(c, xw, rw), f, g);
    collide<R>(k, f, g);
  };

  R cf[kQ], cg[kQ];      // first-step state of row y
  R nf[kQ], ng[kQ];      // first-step state of row y + 1
  R uf[3], ug[3];        // upward populations of row y - 1
  {
    R tf[kQ], tg[kQ];
    first_step(y0 - 1, tf, tg);
    uf[0] = tf[2]; uf[1] = tf[5]; uf[2] = tf[6];
    ug[0] = tg[2]; ug[1] = tg[5]; ug[2] = tg[6];
  }
  first_step(y0, cf, cg);
  if (y0 == 0 && owner && bottom_hot) add_strip_flux<R>(c, k, x, cg);

  for (int y = y0; y < y1; ++y) {
    first_step(y + 1, nf, ng);
    // streamed (pre-collision) state of row y at t+1
    const bool xm_in = c.periodic_x || x - 1 >= 0;
    const bool xp_in = c.periodic_x || x + 1 < c.nx;
    const bool ym_in = c.periodic_y || y - 1 >= 0;
    const bool yp_in = c.periodic_y || y + 1 < c.ny;
    const bool hot = bottom_hot && y == 0;
    R pf[kQ], pg[kQ];
#pragma unroll
    for (int i = 0; i < kQ; ++i) {
      const int ex = cx(i), ey = cy(i);
      R vf, vg;
      if (ey == 0) {
        vf = cf[i];
        vg = cg[i];
      } else if (ey > 0) {
        vf = uf[up_slot(i)];
        vg = ug[up_slot(i)];
      } else {
        vf = nf[i];
        vg = ng[i];
      }
      vf = lane_from(vf, ex);
      vg = lane_from(vg, ex);
      const bool in_x = ex > 0 ? xm_in : (ex < 0 ? xp_in : true);
      const bool in_y = ey > 0 ? ym_in : (ey < 0 ? yp_in : true);
      if (!(in_x && in_y)) {
        // the link crossed a wall: it comes back from the cell itself
        vf = cf[opp(i)];
        vg = cg[opp(i)];
        if (ey == 1 && hot) vg = k.anti(i) - vg;
      }
      pf[i] = vf;
      pg[i] = vg;
    }
    // second step: collide and stream into B
    collide<R>(k, pf, pg);
    if (owner) {
      store_scatter<S, R>(c, k, B, x, y, cell_base(c, x, y), pf, pg);
      if (hot) add_strip_flux<R>(c, k, x, pg);
    }
    // slide the window up by one row
    uf[0] = cf[2]; uf[1] = cf[5]; uf[2] = cf[6];
    ug[0] = cg[2]; ug[1] = cg[5]; ug[2] = cg[6];
#pragma unroll
    for (int i = 0; i < kQ; ++i) {
      cf[i] = nf[i];
      cg[i] = ng[i];
    }
  }
}

template <typename S, typename R, int SEG>
hipError_t dispatch_seg(const CavDev &c, const LaunchCfg &cfg, hipStream_t s) {
  const int strips_x = (c.nx + kStripCols - 1) / kStripCols;
  const int nseg = (c.ny + SEG - 1) / SEG;
  const int waves = strips_x * nseg;
  const int per_block = 4;
  const dim3 grid((waves + per_block - 1) / per_block);
  const int order = (cfg.xcd ? 1 : 0) | (cfg.reverse ? 2 : 0);
  hipLaunchKernelGGL((k_step2<S, R, SEG>), grid, dim3(per_block * kWave), 0, s, c, strips_x,
                     nseg, order);
  return hipGetLastError();
}

template <typename S, typename R>
hipError_t dispatch(const CavDev &c, const LaunchCfg &cfg, hipStream_t s) {
  switch (cfg.seg) {
    case 4: return dispatch_seg<S, R, 4>(c, cfg, s);
    case 8: return dispatch_seg<S, R, 8>(c, cfg, s);
    case 16: return dispatch_seg<S, R, 16>(c, cfg, s);
    case 32: return dispatch_seg<S, R, 32>(c, cfg, s);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace

hipError_t launch_step2(const CavDev &c, int precision, const LaunchCfg &cfg, hipStream_t s) {
  return precision == 0 ? dispatch<double, double>(c, cfg, s) : dispatch<float, float>(c, cfg, s);
}

}  // namespace lbm
