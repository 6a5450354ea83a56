// Single-cavity step kernel: one launch advances one cavity by one time step
// (A-A parity or two-lattice direction from the cavity descriptor).
#include "lbm_device.h"

namespace lbm {
namespace {

using namespace dev;

// Tile of bx x (by*CPL) cells per workgroup; each lane updates CPL cells of
// one column.  order bit 0: consecutive tiles go to one XCD (contiguous bands
// per XCD share its L2 at tile edges); bit 1: walk the tiles backwards on odd
// storage parity.  SM is the storage mode of the launch (update_cell: A-A
// even, A-A odd, two lattices), fixed at compile time so that each instance
// holds the registers of its own path only.
template <typename S, typename R, int CPL, bool NT, int MODEL, int SM>
__global__ __launch_bounds__(256) void k_step(CavDev c, int tiles_x, int order) {
  const int b = tile_of(blockIdx.x, gridDim.x, order & 1, (order & 2) && (c.parity & 1));
  const int tx = b % tiles_x, ty = b / tiles_x;
  const int x = tx * blockDim.x + threadIdx.x;
  const int ybase = ty * blockDim.y * CPL + threadIdx.y;
  const Coef<R> k(c);
  if (x >= c.nx) return;
#pragma unroll
  for (int r = 0; r < CPL; ++r) {
    const int y = ybase + r * blockDim.y;
    if (y < c.ny) update_cell<S, R, MODEL, NT>(c, k, SM, x, y);
  }
}

template <typename S, typename R, bool NT, int MODEL, int SM>
hipError_t dispatch_cpl(const CavDev &c, const LaunchCfg &cfg, hipStream_t s) {
  const int tiles_x = (c.nx + cfg.bx - 1) / cfg.bx;
  const int rows = cfg.by * cfg.cpl;
  const int tiles_y = (c.ny + rows - 1) / rows;
  const dim3 block(cfg.bx, cfg.by);
  const dim3 grid(tiles_x * tiles_y);
  const int order = (cfg.xcd ? 1 : 0) | (cfg.reverse ? 2 : 0);
  switch (cfg.cpl) {
    case 1: hipLaunchKernelGGL((k_step<S, R, 1, NT, MODEL, SM>), grid, block, 0, s, c, tiles_x, order); break;
    case 2: hipLaunchKernelGGL((k_step<S, R, 2, NT, MODEL, SM>), grid, block, 0, s, c, tiles_x, order); break;
    case 4: hipLaunchKernelGGL((k_step<S, R, 4, NT, MODEL, SM>), grid, block, 0, s, c, tiles_x, order); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

template <typename S, typename R, bool NT, int MODEL>
hipError_t dispatch_mode(const CavDev &c, const LaunchCfg &cfg, hipStream_t s) {
  // the storage mode of update_cell: two lattices, or the A-A parity
  if (c.pattern == 1) return dispatch_cpl<S, R, NT, MODEL, 2>(c, cfg, s);
  return c.parity ? dispatch_cpl<S, R, NT, MODEL, 1>(c, cfg, s) : dispatch_cpl<S, R, NT, MODEL, 0>(c, cfg, s);
}

template <typename S, typename R>
hipError_t dispatch(const CavDev &c, const LaunchCfg &cfg, hipStream_t s) {
  return with_model(c.solid_model, [&](auto m) {
    constexpr int M = decltype(m)::value;
    return cfg.nt ? dispatch_mode<S, R, true, M>(c, cfg, s) : dispatch_mode<S, R, false, M>(c, cfg, s);
  });
}

}  // namespace

hipError_t launch_step(const CavDev &c, int precision, const LaunchCfg &cfg, hipStream_t s) {
  return precision == 0 ? dispatch<double, double>(c, cfg, s) : dispatch<float, float>(c, cfg, s);
}

}  // namespace lbm
