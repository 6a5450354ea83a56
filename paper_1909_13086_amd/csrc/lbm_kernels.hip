// gfx950 kernels of the B-TriRT melting step (arXiv 1909.13086).
//
// One lattice update (LU) reads and writes the 9 flow populations f_i and the
// 9 total-enthalpy populations g_i of one cell.  Populations live in 18
// structure-of-arrays planes, x fastest, rows padded to a 64-cell pitch so a
// wavefront covers one contiguous row segment.  Both precisions store the
// populations shifted by their rest state, df_i = f_i - w_i*rho0 and
// dg_i = g_i - w_i*Cp*Tm; the update of Eq. (2) is linear in the
// non-equilibrium part, so it is applied to the shifted values unchanged.
//
// Streaming patterns:
//  - in place ("A-A"): an even step reads a cell's own populations and writes
//    its post-collision values back into the opposite slots of the same cell;
//    an odd step gathers them from the neighbours and scatters the new
//    post-collision values to the neighbours' natural slots.  Each cell reads
//    and writes the same 18 locations, so no two cells touch one location.
//  - two lattices ("A-B"): read the cell's own natural slots from one lattice,
//    scatter to the neighbours in the other.
// Wall rules (Sec. 3.2): a link leaving the cavity returns to the same cell
// (half-way bounce-back: no slip for f, zero flux for g), except that the
// enthalpy links leaving a heated bottom cell through the bottom wall come
// back with the anti-bounce-back value 2 w_i Cp Th - g_i, which holds T = Th
// on the strip.  The strip flux of every step is accumulated per column in
// FP64 so the enthalpy budget closes at any time.
#include "lbm_internal.h"

#include <algorithm>
#include <cmath>

namespace lbm {
namespace {

// D2Q9 velocity set and weights (Sec. 2).
__host__ __device__ constexpr int cx(int i) {
  return i == 1 || i == 5 || i == 8 ? 1 : (i == 3 || i == 6 || i == 7 ? -1 : 0);
}
__host__ __device__ constexpr int cy(int i) {
  return i == 2 || i == 5 || i == 6 ? 1 : (i == 4 || i == 7 || i == 8 ? -1 : 0);
}
__host__ __device__ constexpr int opp(int i) {
  return i == 0 ? 0 : (i <= 4 ? ((i + 1) % 4) + 1 : ((i - 3) % 4) + 5);
}
__host__ __device__ constexpr double wgt(int i) {
  return i == 0 ? 4.0 / 9.0 : (i <= 4 ? 1.0 / 9.0 : 1.0 / 36.0);
}
static_assert(opp(1) == 3 && opp(2) == 4 && opp(3) == 1 && opp(4) == 2, "opp");
static_assert(opp(5) == 7 && opp(6) == 8 && opp(7) == 5 && opp(8) == 6, "opp");

// Rates and constants of one cavity, converted once per thread to the
// arithmetic type R of the update.
template <typename R>
struct Coef {
  R k0g, dk1g, dk2g;       // k0, k1 - k0, k2 - k0 for g
  R k0f, dk1f, dk2f;       // same for f
  R hk1f, hk2f;            // 1 - k1/2, 1 - k2/2 for the force terms
  R Cp, inv_Cp, L, inv_L, rho0, inv_rho0, gb, Tm;
  R c2[3];                 // 2 w_i Cp (Th - Tm) for w = 4/9 (unused), 1/9, 1/36

  __device__ explicit Coef(const CavDev &c) {
    k0g = R(c.k0g);
    dk1g = R(c.k1g - c.k0g);
    dk2g = R(c.k2g - c.k0g);
    k0f = R(c.k0f);
    dk1f = R(c.k1f - c.k0f);
    dk2f = R(c.k2f - c.k0f);
    hk1f = R(1.0 - 0.5 * c.k1f);
    hk2f = R(1.0 - 0.5 * c.k2f);
    Cp = R(c.Cp);
    inv_Cp = R(c.inv_Cp);
    L = R(c.latent);
    inv_L = R(c.inv_latent);
    rho0 = R(c.rho0);
    inv_rho0 = R(c.inv_rho0);
    gb = R(c.gbeta_rho0);
    Tm = R(c.Tm);
    c2[0] = R(2.0 * wgt(0) * c.Cp * c.dT);
    c2[1] = R(2.0 * wgt(1) * c.Cp * c.dT);
    c2[2] = R(2.0 * wgt(5) * c.Cp * c.dT);
  }
  __device__ R anti(int i) const { return i == 0 ? c2[0] : (i <= 4 ? c2[1] : c2[2]); }
};

template <typename R>
__device__ __forceinline__ R sel(bool p, R a, R b) {
  return p ? a : b;
}

// Sec. 2 below Eq. (1): H = Cp T + fl L with isothermal melting at Tm, in
// shifted form dH = H - Cp Tm, theta = T - Tm.
template <typename R>
__device__ __forceinline__ void enthalpy_map(R dH, R L, R inv_L, R inv_Cp, R &fl, R &th) {
  const bool solid = dH <= R(0);
  const bool liquid = !solid && dH >= L;
  fl = solid ? R(0) : (liquid ? R(1) : dH * inv_L);
  th = solid ? dH * inv_Cp : (liquid ? (dH - L) * inv_Cp : R(0));
}

// Relaxation of Eq. (2) written with the combined first- and second-moment
// corrections a1, a2:  p_i <- p_i - k0 (p_i - peq_i) - 3 w_i c_i.a1
//                              - (9/2) w_i (c_i c_i - I/3):a2.
template <typename R>
__device__ __forceinline__ R relax_one(int i, R p, R peq, R k0, R a1x, R a1y, R a2xx, R a2xy,
                                       R a2yy) {
  constexpr R third = R(1.0 / 3.0);
  const R w = R(wgt(i));
  const R ex = R(cx(i)), ey = R(cy(i));
  const R c1 = ex * a1x + ey * a1y;
  const R qa = (ex * ex - third) * a2xx + R(2) * ex * ey * a2xy + (ey * ey - third) * a2yy;
  return p - k0 * (p - peq) - R(3) * w * c1 - R(4.5) * w * qa;
}

// One B-TriRT collision of a cell, shifted populations in place.  Returns
// nothing; fl/theta/ux/uy are the pre-collision macroscopic values.
template <typename R>
__device__ __forceinline__ void collide(const Coef<R> &k, R (&f)[kQ], R (&g)[kQ]) {
  constexpr R third = R(1.0 / 3.0);
  // (a) total enthalpy
  const R dH = ((g[0] + g[1]) + (g[2] + g[3])) + ((g[4] + g[5]) + (g[6] + g[7])) + g[8];
  // (b) temperature and liquid fraction
  R fl, th;
  enthalpy_map(dH, k.L, k.inv_L, k.inv_Cp, fl, th);
  // (c) flow moments, buoyancy, velocity immobilised in the solid
  const R drho = ((f[0] + f[1]) + (f[2] + f[3])) + ((f[4] + f[5]) + (f[6] + f[7])) + f[8];
  const R jx = (f[1] - f[3]) + (f[5] - f[6]) + (f[8] - f[7]);
  const R jy = (f[2] - f[4]) + (f[5] + f[6]) - (f[7] + f[8]);
  const R Fy = k.gb * th;
  const R ux = fl * jx * k.inv_rho0;
  const R uy = fl * (jy + R(0.5) * Fy) * k.inv_rho0;
  // (d) flow collision with the Hermite-projected force
  {
    const R d = (f[5] + f[6]) + (f[7] + f[8]);
    const R pxx = (f[1] + f[3]) + d;
    const R pyy = (f[2] + f[4]) + d;
    const R pxy = (f[5] - f[6]) + (f[7] - f[8]);
    const R r3 = drho * third;
    const R m1x = jx - k.rho0 * ux, m1y = jy - k.rho0 * uy;
    const R m2xx = pxx - (r3 + k.rho0 * ux * ux);
    const R m2yy = pyy - (r3 + k.rho0 * uy * uy);
    const R m2xy = pxy - k.rho0 * ux * uy;
    const R a1x = k.dk1f * m1x;
    const R a1y = k.dk1f * m1y - k.hk1f * Fy;
    const R a2xx = k.dk2f * m2xx;
    const R a2xy = k.dk2f * m2xy - k.hk2f * (ux * Fy);
    const R a2yy = k.dk2f * m2yy - k.hk2f * (R(2) * uy * Fy);
    const R uu15 = R(1.5) * (ux * ux + uy * uy);
#pragma unroll
    for (int i = 0; i < kQ; ++i) {
      const R cu = R(cx(i)) * ux + R(cy(i)) * uy;
      const R feq = R(wgt(i)) * (drho + k.rho0 * (R(3) * cu + R(4.5) * cu * cu - uu15));
      f[i] = relax_one<R>(i, f[i], feq, k.k0f, a1x, a1y, a2xx, a2xy, a2yy);
    }
  }
  // (e) enthalpy collision with the equilibrium of Eq. (3)
  {
    const R T = k.Tm + th;
    const R CpT = k.Cp * T;
    const R Cpth = k.Cp * th;
    const R d = (g[5] + g[6]) + (g[7] + g[8]);
    const R gx = (g[1] - g[3]) + (g[5] - g[6]) + (g[8] - g[7]);
    const R gy = (g[2] - g[4]) + (g[5] + g[6]) - (g[7] + g[8]);
    const R qxx = (g[1] + g[3]) + d;
    const R qyy = (g[2] + g[4]) + d;
    const R qxy = (g[5] - g[6]) + (g[7] - g[8]);
    const R a1x = k.dk1g * (gx - CpT * ux);
    const R a1y = k.dk1g * (gy - CpT * uy);
    const R a2xx = k.dk2g * (qxx - Cpth * third);
    const R a2xy = k.dk2g * qxy;
    const R a2yy = k.dk2g * (qyy - Cpth * third);
#pragma unroll
    for (int i = 0; i < kQ; ++i) {
      R geq;
      if (i == 0) {
        geq = dH - Cpth + R(wgt(0)) * Cpth;
      } else {
        const R cu = R(cx(i)) * ux + R(cy(i)) * uy;
        geq = R(wgt(i)) * Cpth + R(3) * R(wgt(i)) * CpT * cu;
      }
      g[i] = relax_one<R>(i, g[i], geq, k.k0g, a1x, a1y, a2xx, a2xy, a2yy);
    }
  }
}

// Neighbour addressing of cell (x, y): index of the cell one link away in
// direction (dx, dy) and whether it exists (periodic sides wrap).
struct Nbr {
  int64_t idx[9];   // indexed by population number of the direction
  bool in[9];
};

__device__ __forceinline__ void neighbours(const CavDev &c, int x, int y, int sign, Nbr &n) {
  const int xm = x - 1, xp = x + 1, ym = y - 1, yp = y + 1;
  const bool xm_in = c.periodic_x || xm >= 0;
  const bool xp_in = c.periodic_x || xp < c.nx;
  const bool ym_in = c.periodic_y || ym >= 0;
  const bool yp_in = c.periodic_y || yp < c.ny;
  const int xmw = xm < 0 ? xm + c.nx : xm;
  const int xpw = xp >= c.nx ? xp - c.nx : xp;
  const int ymw = ym < 0 ? ym + c.ny : ym;
  const int ypw = yp >= c.ny ? yp - c.ny : yp;
#pragma unroll
  for (int i = 0; i < kQ; ++i) {
    const int ex = sign * cx(i), ey = sign * cy(i);
    const int nx_ = ex < 0 ? xmw : (ex > 0 ? xpw : x);
    const int ny_ = ey < 0 ? ymw : (ey > 0 ? ypw : y);
    const bool ix = ex < 0 ? xm_in : (ex > 0 ? xp_in : true);
    const bool iy = ey < 0 ? ym_in : (ey > 0 ? yp_in : true);
    n.in[i] = ix && iy;
    n.idx[i] = (int64_t)ny_ * c.pitch + nx_;
  }
}

__device__ __forceinline__ bool heated(const CavDev &c, int x, int y) {
  return y == 0 && x >= c.hlo && x <= c.hhi;
}

// Natural pre-collision populations of a cell (state of A-A parity 0, or of
// the current lattice of the two-lattice pattern).
template <typename S, typename R>
__device__ __forceinline__ void load_natural(const S *__restrict__ P, int64_t plane, int64_t idx,
                                             R (&f)[kQ], R (&g)[kQ]) {
#pragma unroll
  for (int i = 0; i < kQ; ++i) {
    f[i] = R(P[i * plane + idx]);
    g[i] = R(P[(kQ + i) * plane + idx]);
  }
}

// Pre-collision populations gathered from the neighbours' swapped slots
// (A-A parity 1); links from outside come back from the cell's own slot.
template <typename S, typename R>
__device__ __forceinline__ void load_gather(const CavDev &c, const Coef<R> &k,
                                            const S *__restrict__ P, int x, int y, int64_t idx,
                                            R (&f)[kQ], R (&g)[kQ]) {
  Nbr n;
  neighbours(c, x, y, -1, n);
  const bool bottom_hot = !c.periodic_y && heated(c, x, y);
#pragma unroll
  for (int i = 0; i < kQ; ++i) {
    const int64_t src = n.in[i] ? opp(i) * c.plane + n.idx[i] : i * c.plane + idx;
    f[i] = R(P[src]);
    R v = R(P[kQ * c.plane + src]);
    if (cy(i) == 1 && bottom_hot && !n.in[i]) v = k.anti(i) - v;
    g[i] = v;
  }
}

// Post-collision populations scattered to the neighbours' natural slots;
// links leaving the cavity are reflected into the cell's opposite slot.
template <typename S, typename R>
__device__ __forceinline__ void store_scatter(const CavDev &c, const Coef<R> &k,
                                              S *__restrict__ P, int x, int y, int64_t idx,
                                              const R (&f)[kQ], const R (&g)[kQ]) {
  Nbr n;
  neighbours(c, x, y, +1, n);
  const bool bottom_hot = !c.periodic_y && heated(c, x, y);
#pragma unroll
  for (int i = 0; i < kQ; ++i) {
    const int64_t dst = n.in[i] ? i * c.plane + n.idx[i] : opp(i) * c.plane + idx;
    P[dst] = S(f[i]);
    R v = g[i];
    if (cy(i) == -1 && bottom_hot && !n.in[i]) v = k.anti(i) - v;
    P[kQ * c.plane + dst] = S(v);
  }
}

template <typename S, typename R>
__device__ __forceinline__ void store_swapped(S *__restrict__ P, int64_t plane, int64_t idx,
                                              const R (&f)[kQ], const R (&g)[kQ]) {
#pragma unroll
  for (int i = 0; i < kQ; ++i) {
    P[opp(i) * plane + idx] = S(f[i]);
    P[(kQ + opp(i)) * plane + idx] = S(g[i]);
  }
}

// Strip enthalpy that the post-collision state of a heated bottom cell sends
// back in the next step: each of its three upward links returns with
// 2 w Cp (Th - Tm) - g_down, and adds twice its excess over w Cp (Th - Tm).
template <typename R>
__device__ __forceinline__ void add_strip_flux(const CavDev &c, const Coef<R> &k, int x,
                                               const R (&g)[kQ]) {
  double q = 0.0;
#pragma unroll
  for (int i = 0; i < kQ; ++i) {
    if (cy(i) != -1) continue;
    const R gin = k.anti(i) - g[i];
    q += 2.0 * ((double)gin - wgt(i) * c.Cp * c.dT);
  }
  c.cumq[x] += q;
}

// One lattice update of cell (x, y) for the given storage mode.
//   mode 0: A-A even, mode 1: A-A odd, mode 2: two lattices (src -> dst)
template <typename S, typename R>
__device__ __forceinline__ void update_cell(const CavDev &c, const Coef<R> &k, int mode, int x,
                                            int y) {
  const int64_t idx = (int64_t)y * c.pitch + x;
  R f[kQ], g[kQ];
  if (mode == 0) {
    S *P = static_cast<S *>(c.pop[0]);
    load_natural<S, R>(P, c.plane, idx, f, g);
    collide<R>(k, f, g);
    store_swapped<S, R>(P, c.plane, idx, f, g);
  } else if (mode == 1) {
    S *P = static_cast<S *>(c.pop[0]);
    load_gather<S, R>(c, k, P, x, y, idx, f, g);
    collide<R>(k, f, g);
    store_scatter<S, R>(c, k, P, x, y, idx, f, g);
  } else {
    const S *A = static_cast<const S *>(c.parity ? c.pop[1] : c.pop[0]);
    S *B = static_cast<S *>(c.parity ? c.pop[0] : c.pop[1]);
    load_natural<S, R>(A, c.plane, idx, f, g);
    collide<R>(k, f, g);
    store_scatter<S, R>(c, k, B, x, y, idx, f, g);
  }
  if (!c.periodic_y && heated(c, x, y)) add_strip_flux<R>(c, k, x, g);
}

__device__ __forceinline__ int storage_mode(const CavDev &c) {
  return c.pattern == 1 ? 2 : c.parity;
}

// Spread consecutive workgroup ids over the 8 XCDs so that each XCD gets a
// contiguous band of tiles (workgroups are dispatched round-robin over XCDs).
__device__ __forceinline__ int xcd_band(int b, int nb) {
  const int xcd = b % kXcds, local = b / kXcds;
  const int q = nb / kXcds, r = nb % kXcds;
  return xcd < r ? xcd * (q + 1) + local : r * (q + 1) + (xcd - r) * q + local;
}

template <typename S, typename R, int CPL>
__global__ __launch_bounds__(256) void k_step(CavDev c, int tiles_x, int xcd) {
  const int b = xcd ? xcd_band(blockIdx.x, gridDim.x) : (int)blockIdx.x;
  const int tx = b % tiles_x, ty = b / tiles_x;
  const int x = tx * blockDim.x + threadIdx.x;
  const int ybase = ty * blockDim.y * CPL + threadIdx.y;
  const Coef<R> k(c);
  const int mode = storage_mode(c);
  if (x >= c.nx) return;
#pragma unroll
  for (int r = 0; r < CPL; ++r) {
    const int y = ybase + r * blockDim.y;
    if (y < c.ny) update_cell<S, R>(c, k, mode, x, y);
  }
}

// Batched step over tiles of many cavities.  hdr holds {first tile, tile
// count} of this launch, read on the device so that a captured launch stays
// valid when cavities join or leave.  The tile list is cut into 8 contiguous
// bands, one per XCD (workgroups are dispatched round-robin over the XCDs),
// and each XCD's workgroups stride through its band, so neighbouring tiles
// share that XCD's L2.  Cavity j advances in this launch only while
// launch_index < active_steps(j); its storage parity is its chunk-start
// parity flipped by the launch index.
template <typename S, typename R>
__global__ __launch_bounds__(256) void k_step_batch(const CavDev *__restrict__ cavs,
                                                    const BatchTile *__restrict__ tiles,
                                                    const int32_t *__restrict__ hdr,
                                                    int tile_cap, int tile_rows,
                                                    int launch_index) {
  const int first = hdr[0], ntiles = hdr[1];
  if (first < 0 || ntiles <= 0 || first > tile_cap - ntiles) return;
  const int xcd = blockIdx.x % kXcds, lb = blockIdx.x / kXcds;
  const int nbx = (gridDim.x - xcd + kXcds - 1) / kXcds;
  const int t0 = (int)((int64_t)ntiles * xcd / kXcds);
  const int t1 = (int)((int64_t)ntiles * (xcd + 1) / kXcds);
  for (int t = t0 + lb; t < t1; t += nbx) {
    const BatchTile tile = tiles[first + t];
    CavDev c = cavs[tile.cav];
    if (launch_index >= c.active_steps) continue;
    c.parity ^= (launch_index & 1);
    const Coef<R> k(c);
    const int mode = storage_mode(c);
    const int x = tile.x0 + threadIdx.x;
    if (x >= c.nx) continue;
    for (int r = threadIdx.y; r < tile_rows; r += blockDim.y) {
      const int y = tile.y0 + r;
      if (y < c.ny) update_cell<S, R>(c, k, mode, x, y);
    }
  }
}

// ---- initial state, load/save, fields and reductions -----------------------

// State at rest from a temperature: liquid where T > Tm, g at the equilibrium
// of Eq. (3) with u = 0, f_i = w_i rho0 (shifted: df = 0).
template <typename S>
__global__ void k_init(CavDev c, int mode, double T0, double amp, double sigma) {
  const int x = blockIdx.x * blockDim.x + threadIdx.x;
  const int y = blockIdx.y;
  if (x >= c.nx || y >= c.ny) return;
  double T = c.Tm;
  if (mode == 1) {
    T = T0;
  } else if (mode == 2) {
    const double dx = (x + 0.5) - 0.5 * c.nx, dy = (y + 0.5) - 0.5 * c.ny;
    T = T0 + amp * exp(-(dx * dx + dy * dy) / (2.0 * sigma * sigma));
  }
  const double fl = T > c.Tm ? 1.0 : 0.0;
  const double th = T - c.Tm;
  const double dH = c.Cp * th + fl * c.latent;
  const int64_t idx = (int64_t)y * c.pitch + x;
  S *P = static_cast<S *>(c.pop[0]);
#pragma unroll
  for (int i = 0; i < kQ; ++i) {
    P[i * c.plane + idx] = S(0);
    const double geq = i == 0 ? dH - c.Cp * th + wgt(0) * c.Cp * th : wgt(i) * c.Cp * th;
    P[(kQ + i) * c.plane + idx] = S(geq);
  }
}

template <typename S>
__global__ void k_load(CavDev c, const double *__restrict__ f, const double *__restrict__ g) {
  const int x = blockIdx.x * blockDim.x + threadIdx.x;
  const int y = blockIdx.y;
  if (x >= c.nx || y >= c.ny) return;
  const int64_t n = (int64_t)c.nx * c.ny, h = (int64_t)y * c.nx + x;
  const int64_t idx = (int64_t)y * c.pitch + x;
  S *P = static_cast<S *>(c.pop[0]);
#pragma unroll
  for (int i = 0; i < kQ; ++i) {
    P[i * c.plane + idx] = S(f[i * n + h] - wgt(i) * c.rho0);
    P[(kQ + i) * c.plane + idx] = S(g[i * n + h] - wgt(i) * c.Cp * c.Tm);
  }
}

// Pre-collision shifted populations of cell (x, y) in the storage type,
// converted to double afterwards (the anti-bounce-back value is formed in
// the storage precision as the update forms it).
template <typename S>
__device__ __forceinline__ void load_pre(const CavDev &c, int x, int y, double (&f)[kQ],
                                         double (&g)[kQ]) {
  using R = S;
  const int64_t idx = (int64_t)y * c.pitch + x;
  R fr[kQ], gr[kQ];
  if (c.pattern == 1) {
    load_natural<S, R>(static_cast<const S *>(c.parity ? c.pop[1] : c.pop[0]), c.plane, idx, fr,
                       gr);
  } else if (c.parity == 0) {
    load_natural<S, R>(static_cast<const S *>(c.pop[0]), c.plane, idx, fr, gr);
  } else {
    const Coef<R> k(c);
    load_gather<S, R>(c, k, static_cast<const S *>(c.pop[0]), x, y, idx, fr, gr);
  }
#pragma unroll
  for (int i = 0; i < kQ; ++i) {
    f[i] = (double)fr[i];
    g[i] = (double)gr[i];
  }
}

template <typename S>
__global__ void k_save(CavDev c, double *__restrict__ f, double *__restrict__ g) {
  const int x = blockIdx.x * blockDim.x + threadIdx.x;
  const int y = blockIdx.y;
  if (x >= c.nx || y >= c.ny) return;
  const int64_t n = (int64_t)c.nx * c.ny, h = (int64_t)y * c.nx + x;
  double fd[kQ], gd[kQ];
  load_pre<S>(c, x, y, fd, gd);
#pragma unroll
  for (int i = 0; i < kQ; ++i) {
    f[i * n + h] = fd[i] + wgt(i) * c.rho0;
    g[i * n + h] = gd[i] + wgt(i) * c.Cp * c.Tm;
  }
}

struct Macro {
  double T, fl, H, ux, uy, rho;
};

// Macroscopic values of a pre-collision cell, FP64 (steps (a)-(c) of the update).
__device__ __forceinline__ Macro macros(const CavDev &c, const double (&f)[kQ],
                                        const double (&g)[kQ]) {
  Macro m;
  double dH = 0.0, drho = 0.0, jx = 0.0, jy = 0.0;
#pragma unroll
  for (int i = 0; i < kQ; ++i) {
    dH += g[i];
    drho += f[i];
    jx += cx(i) * f[i];
    jy += cy(i) * f[i];
  }
  double fl, th;
  enthalpy_map<double>(dH, c.latent, c.inv_latent, c.inv_Cp, fl, th);
  const double Fy = c.gbeta_rho0 * th;
  m.T = c.Tm + th;
  m.fl = fl;
  m.H = dH + c.Cp * c.Tm;
  m.ux = fl * jx * c.inv_rho0;
  m.uy = fl * (jy + 0.5 * Fy) * c.inv_rho0;
  m.rho = c.rho0 + drho;
  return m;
}

template <typename S>
__global__ void k_fields(CavDev c, uint32_t mask, double *__restrict__ out) {
  const int x = blockIdx.x * blockDim.x + threadIdx.x;
  const int y = blockIdx.y;
  if (x >= c.nx || y >= c.ny) return;
  const int64_t n = (int64_t)c.nx * c.ny, h = (int64_t)y * c.nx + x;
  double f[kQ], g[kQ];
  load_pre<S>(c, x, y, f, g);
  const Macro m = macros(c, f, g);
  const double v[6] = {m.T, m.fl, m.H, m.ux, m.uy, m.rho};
  int slot = 0;
#pragma unroll
  for (int b = 0; b < 6; ++b) {
    if (mask & (1u << b)) {
      out[slot * n + h] = v[b];
      ++slot;
    }
  }
}

// Compensated (sum, correction) pair: Knuth's TwoSum keeps the rounding error
// of each addition, so sums of the same values in the same tree order are
// reproducible and accurate to ~1 ulp of the result.
struct CSum {
  double s, c;
};
__device__ __forceinline__ void cs_add(CSum &a, double x) {
  const double t = a.s + x;
  const double bp = t - a.s;
  a.c += (a.s - (t - bp)) + (x - bp);
  a.s = t;
}
__device__ __forceinline__ CSum cs_merge(CSum a, CSum b) {
  const double t = a.s + b.s;
  const double bp = t - a.s;
  const double e = (a.s - (t - bp)) + (b.s - bp);
  return CSum{t, a.c + b.c + e};
}

constexpr int kNSum = 4;  // fl, H, rho, strip flux

struct RedAcc {
  CSum sum[kNSum];
  double umax2;
  double nonfinite;
};

__device__ __forceinline__ void acc_init(RedAcc &a) {
#pragma unroll
  for (int k = 0; k < kNSum; ++k) a.sum[k] = CSum{0.0, 0.0};
  a.umax2 = 0.0;
  a.nonfinite = 0.0;
}

__device__ __forceinline__ void acc_merge(RedAcc &a, const RedAcc &b) {
#pragma unroll
  for (int k = 0; k < kNSum; ++k) a.sum[k] = cs_merge(a.sum[k], b.sum[k]);
  a.umax2 = fmax(a.umax2, b.umax2);
  a.nonfinite += b.nonfinite;
}

// Wavefront (64 lanes) then workgroup reduction in a fixed tree order.
__device__ void block_reduce(RedAcc &a, RedAcc *lds) {
#pragma unroll
  for (int off = kWave / 2; off > 0; off >>= 1) {
    RedAcc o;
#pragma unroll
    for (int k = 0; k < kNSum; ++k) {
      o.sum[k].s = __shfl_down(a.sum[k].s, off, kWave);
      o.sum[k].c = __shfl_down(a.sum[k].c, off, kWave);
    }
    o.umax2 = __shfl_down(a.umax2, off, kWave);
    o.nonfinite = __shfl_down(a.nonfinite, off, kWave);
    acc_merge(a, o);
  }
  const int lane = threadIdx.x % kWave, wave = threadIdx.x / kWave;
  if (lane == 0) lds[wave] = a;
  __syncthreads();
  if (threadIdx.x == 0) {
    const int nw = (blockDim.x + kWave - 1) / kWave;
    for (int w = 1; w < nw; ++w) acc_merge(a, lds[w]);
  }
}

constexpr int kPartialStride = 2 * kNSum + 2;

template <typename S>
__global__ __launch_bounds__(kRedThreads) void k_reduce(CavDev c, double *__restrict__ partials) {
  __shared__ RedAcc lds[kRedThreads / kWave];
  RedAcc a;
  acc_init(a);
  const int64_t n = (int64_t)c.nx * c.ny;
  for (int64_t cell = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; cell < n;
       cell += (int64_t)gridDim.x * blockDim.x) {
    const int y = (int)(cell / c.nx), x = (int)(cell % c.nx);
    double f[kQ], g[kQ];
    load_pre<S>(c, x, y, f, g);
    bool fin = true;
#pragma unroll
    for (int i = 0; i < kQ; ++i) fin = fin && isfinite(f[i]) && isfinite(g[i]);
    if (!fin) a.nonfinite += 1.0;
    const Macro m = macros(c, f, g);
    cs_add(a.sum[0], m.fl);
    cs_add(a.sum[1], m.H);
    cs_add(a.sum[2], m.rho);
    a.umax2 = fmax(a.umax2, m.ux * m.ux + m.uy * m.uy);
    if (!c.periodic_y && heated(c, x, y)) {
#pragma unroll
      for (int i = 0; i < kQ; ++i) {
        if (cy(i) != 1) continue;
        cs_add(a.sum[3], 2.0 * (g[i] - wgt(i) * c.Cp * c.dT));
      }
    }
  }
  block_reduce(a, lds);
  if (threadIdx.x == 0) {
    double *p = partials + (int64_t)blockIdx.x * kPartialStride;
#pragma unroll
    for (int k = 0; k < kNSum; ++k) {
      p[2 * k] = a.sum[k].s;
      p[2 * k + 1] = a.sum[k].c;
    }
    p[2 * kNSum] = a.umax2;
    p[2 * kNSum + 1] = a.nonfinite;
  }
}

__global__ __launch_bounds__(kRedThreads) void k_reduce_final(CavDev c,
                                                              const double *__restrict__ partials,
                                                              int nblocks, StatsDev *out) {
  __shared__ RedAcc lds[kRedThreads / kWave];
  RedAcc a;
  acc_init(a);
  for (int b = threadIdx.x; b < nblocks; b += blockDim.x) {
    const double *p = partials + (int64_t)b * kPartialStride;
    RedAcc o;
#pragma unroll
    for (int k = 0; k < kNSum; ++k) o.sum[k] = CSum{p[2 * k], p[2 * k + 1]};
    o.umax2 = p[2 * kNSum];
    o.nonfinite = p[2 * kNSum + 1];
    acc_merge(a, o);
  }
  // strip enthalpy of every step so far, summed over the heated columns
  CSum qcum{0.0, 0.0};
  if (c.hlo <= c.hhi) {
    for (int x = c.hlo + threadIdx.x; x <= c.hhi; x += blockDim.x) cs_add(qcum, c.cumq[x]);
  }
  block_reduce(a, lds);
  __syncthreads();
  // second pass for qcum, reusing the accumulator layout
  RedAcc qa;
  acc_init(qa);
  qa.sum[0] = qcum;
  block_reduce(qa, lds);
  if (threadIdx.x == 0) {
    const double n = (double)c.nx * (double)c.ny;
    out->melt_fraction = (a.sum[0].s + a.sum[0].c) / n;
    out->total_H = a.sum[1].s + a.sum[1].c;
    out->mass = a.sum[2].s + a.sum[2].c;
    out->heater_q = a.sum[3].s + a.sum[3].c;
    out->max_u = sqrt(a.umax2);
    out->nonfinite = a.nonfinite;
    out->heat_in_cum = qa.sum[0].s + qa.sum[0].c;
    out->pad = 0.0;
  }
}

__global__ void k_fill_zero(uint32_t *p, size_t n) {
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (size_t)gridDim.x * blockDim.x)
    p[i] = 0u;
}

__global__ void k_copy_stats(const StatsDev *src, StatsDev *dst) {
  if (threadIdx.x == 0) *dst = *src;
}

template <typename S, typename R>
hipError_t step_dispatch(const CavDev &c, const LaunchCfg &cfg, hipStream_t s) {
  const int tiles_x = (c.nx + cfg.bx - 1) / cfg.bx;
  const int rows = cfg.by * cfg.cpl;
  const int tiles_y = (c.ny + rows - 1) / rows;
  const dim3 block(cfg.bx, cfg.by);
  const dim3 grid(tiles_x * tiles_y);
  switch (cfg.cpl) {
    case 1: hipLaunchKernelGGL((k_step<S, R, 1>), grid, block, 0, s, c, tiles_x, cfg.xcd); break;
    case 2: hipLaunchKernelGGL((k_step<S, R, 2>), grid, block, 0, s, c, tiles_x, cfg.xcd); break;
    case 4: hipLaunchKernelGGL((k_step<S, R, 4>), grid, block, 0, s, c, tiles_x, cfg.xcd); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

}  // namespace

hipError_t launch_step(const CavDev &c, int precision, const LaunchCfg &cfg, hipStream_t s) {
  return precision == 0 ? step_dispatch<double, double>(c, cfg, s)
                        : step_dispatch<float, float>(c, cfg, s);
}

hipError_t launch_step_batch(const CavDev *cavs_dev, const BatchTile *tiles_dev,
                             const int32_t *hdr_dev, int tile_cap, int precision, int tile_bx,
                             int tile_rows, int launch_index, int grid, hipStream_t s) {
  const int by = 256 / tile_bx;
  const dim3 block(tile_bx, by < 1 ? 1 : by);
  if (precision == 0)
    hipLaunchKernelGGL((k_step_batch<double, double>), dim3(grid), block, 0, s, cavs_dev,
                       tiles_dev, hdr_dev, tile_cap, tile_rows, launch_index);
  else
    hipLaunchKernelGGL((k_step_batch<float, float>), dim3(grid), block, 0, s, cavs_dev,
                       tiles_dev, hdr_dev, tile_cap, tile_rows, launch_index);
  return hipGetLastError();
}

static dim3 row_grid(const CavDev &c, int bx) { return dim3((c.nx + bx - 1) / bx, c.ny); }

hipError_t launch_init(const CavDev &c, int precision, int mode, double T0, double amp,
                       double sigma, hipStream_t s) {
  if (precision == 0)
    hipLaunchKernelGGL(k_init<double>, row_grid(c, 64), dim3(64), 0, s, c, mode, T0, amp, sigma);
  else
    hipLaunchKernelGGL(k_init<float>, row_grid(c, 64), dim3(64), 0, s, c, mode, T0, amp, sigma);
  return hipGetLastError();
}

hipError_t launch_load(const CavDev &c, int precision, const double *f, const double *g,
                       hipStream_t s) {
  if (precision == 0)
    hipLaunchKernelGGL(k_load<double>, row_grid(c, 64), dim3(64), 0, s, c, f, g);
  else
    hipLaunchKernelGGL(k_load<float>, row_grid(c, 64), dim3(64), 0, s, c, f, g);
  return hipGetLastError();
}

hipError_t launch_save(const CavDev &c, int precision, double *f, double *g, hipStream_t s) {
  if (precision == 0)
    hipLaunchKernelGGL(k_save<double>, row_grid(c, 64), dim3(64), 0, s, c, f, g);
  else
    hipLaunchKernelGGL(k_save<float>, row_grid(c, 64), dim3(64), 0, s, c, f, g);
  return hipGetLastError();
}

hipError_t launch_fields(const CavDev &c, int precision, uint32_t mask, double *out,
                         hipStream_t s) {
  if (precision == 0)
    hipLaunchKernelGGL(k_fields<double>, row_grid(c, 64), dim3(64), 0, s, c, mask, out);
  else
    hipLaunchKernelGGL(k_fields<float>, row_grid(c, 64), dim3(64), 0, s, c, mask, out);
  return hipGetLastError();
}

hipError_t launch_reduce(const CavDev &c, int precision, double *partials, StatsDev *out,
                         hipStream_t s) {
  if (precision == 0)
    hipLaunchKernelGGL(k_reduce<double>, dim3(kRedBlocks), dim3(kRedThreads), 0, s, c, partials);
  else
    hipLaunchKernelGGL(k_reduce<float>, dim3(kRedBlocks), dim3(kRedThreads), 0, s, c, partials);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_reduce_final, dim3(1), dim3(kRedThreads), 0, s, c, partials, kRedBlocks,
                     out);
  return hipGetLastError();
}

hipError_t launch_fill_zero(void *p, size_t bytes, hipStream_t s) {
  if (bytes == 0) return hipSuccess;
  const size_t n = bytes / 4;
  const int blocks = (int)std::min<size_t>((n + 255) / 256, 4096);
  hipLaunchKernelGGL(k_fill_zero, dim3(blocks), dim3(256), 0, s, static_cast<uint32_t *>(p), n);
  return hipGetLastError();
}

hipError_t launch_copy_stats(const StatsDev *src, StatsDev *dst, hipStream_t s) {
  hipLaunchKernelGGL(k_copy_stats, dim3(1), dim3(64), 0, s, src, dst);
  return hipGetLastError();
}

}  // namespace lbm
