// Device code shared by the gfx950 kernels of the B-TriRT melting step
// (arXiv 1909.13086).
//
// One lattice update (LU) reads and writes the 9 flow populations f_i and the
// 9 total-enthalpy populations g_i of one cell.  Populations live in 18
// structure-of-arrays planes, blocked by 64-cell row chunks (cell_base), rows
// padded to a 64-cell pitch so a wavefront covers one chunk.  Both precisions
// store the populations shifted by their rest state, df_i = f_i - w_i*rho0
// and dg_i = g_i - w_i*Cp*Tm; the update of Eq. (2) is linear in the
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
#pragma once

#include "lbm_internal.h"

#include <algorithm>
#include <cmath>
#include <type_traits>

namespace lbm {
namespace dev {



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
  R omk0g, omk0f;          // 1 - k0
  R hk1f, hk2f;            // 1 - k1/2, 1 - k2/2 for the force terms
  R Cp, inv_Cp, L, inv_L, rho0, inv_rho0, gb, Tm;
  R c2[3];                 // 2 w_i Cp (Th - Tm) for w = 4/9 (unused), 1/9, 1/36
  R darcy_c, darcy_eps;    // drag constants of the Darcy solid model

  __device__ explicit Coef(const CavDev &c) {
    k0g = R(c.k0g);
    dk1g = R(c.k1g - c.k0g);
    dk2g = R(c.k2g - c.k0g);
    k0f = R(c.k0f);
    dk1f = R(c.k1f - c.k0f);
    dk2f = R(c.k2f - c.k0f);
    omk0g = R(1.0 - c.k0g);
    omk0f = R(1.0 - c.k0f);
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
    darcy_c = R(c.darcy_c);
    darcy_eps = R(c.darcy_eps);
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

// Relaxation of Eq. (2) for a pair of opposite populations (i, opp(i)).
// With the combined first- and second-moment corrections a1, a2, Eq. (2)
// reads p_i* = p_i - k0 (p_i - peq_i) - 3 w_i c_i.a1 - (9/2) w_i Q_i:a2,
// Q_i = c_i c_i - I/3.  Under c -> -c the equilibrium splits into an even
// part E and an odd part O, c.a1 changes sign and Q:a2 does not, so
//   p_{+/-}* = (1 - k0) p_{+/-} + (k0 E - t2) +/- (k0 O - t1)
// with t1 = 3 w c.a1 and t2 = (9/2) w Q:a2 taken for the "+" member.
template <typename R>
__device__ __forceinline__ void relax_pair(R &pp, R &pm, R omk0, R k0, R E, R O, R t1, R t2) {
  const R even = k0 * E - t2;
  const R odd = k0 * O - t1;
  pp = omk0 * pp + (even + odd);
  pm = omk0 * pm + (even - odd);
}

// The same followed by partial bounce-back with solid fraction ns: each
// member mixes its post-collision value with its partner's pre-collision one.
template <typename R>
__device__ __forceinline__ void relax_pair_pbb(R &pp, R &pm, R omk0, R k0, R E, R O, R t1, R t2,
                                               R ns) {
  const R pp0 = pp, pm0 = pm;
  relax_pair<R>(pp, pm, omk0, k0, E, O, t1, t2);
  pp = (R(1) - ns) * pp + ns * pm0;
  pm = (R(1) - ns) * pm + ns * pp0;
}

// The four pairs of D2Q9 directions, "+" member first: (1, 3) along x,
// (2, 4) along y, (5, 7) along (1, 1), (6, 8) along (-1, 1).  For each pair,
// c.u, c.a1 and Q:a2 of the "+" member.
template <typename R>
struct PairTerms {
  R cu[4], c1[4], qa[4];
  __device__ PairTerms(R ux, R uy, R a1x, R a1y, R a2xx, R a2xy, R a2yy) {
    constexpr R third = R(1.0 / 3.0), two_thirds = R(2.0 / 3.0);
    cu[0] = ux;
    cu[1] = uy;
    cu[2] = ux + uy;
    cu[3] = uy - ux;
    c1[0] = a1x;
    c1[1] = a1y;
    c1[2] = a1x + a1y;
    c1[3] = a1y - a1x;
    const R d = two_thirds * (a2xx + a2yy);
    qa[0] = two_thirds * a2xx - third * a2yy;
    qa[1] = two_thirds * a2yy - third * a2xx;
    qa[2] = d + R(2) * a2xy;
    qa[3] = d - R(2) * a2xy;
  }
};
__device__ constexpr int pair_plus(int p) { return p == 0 ? 1 : (p == 1 ? 2 : (p == 2 ? 5 : 6)); }
__device__ constexpr int pair_minus(int p) { return p == 0 ? 3 : (p == 1 ? 4 : (p == 2 ? 7 : 8)); }
__device__ constexpr double pair_w(int p) { return p < 2 ? 1.0 / 9.0 : 1.0 / 36.0; }

// One B-TriRT collision of a cell, shifted populations in place.  MODEL is
// the solid-phase treatment of the flow (kSolid*), fixed at compile time.
template <typename R, int MODEL>
__device__ __forceinline__ void collide(const Coef<R> &k, R (&f)[kQ], R (&g)[kQ]) {
  constexpr R third = R(1.0 / 3.0);
  constexpr R w0 = R(4.0 / 9.0);
  // (a) total enthalpy
  const R dH = ((g[0] + g[1]) + (g[2] + g[3])) + ((g[4] + g[5]) + (g[6] + g[7])) + g[8];
  // (b) temperature and liquid fraction
  R fl, th;
  enthalpy_map(dH, k.L, k.inv_L, k.inv_Cp, fl, th);
  // (c) flow moments, buoyancy, velocity immobilised in the solid
  const R drho = ((f[0] + f[1]) + (f[2] + f[3])) + ((f[4] + f[5]) + (f[6] + f[7])) + f[8];
  const R jx = (f[1] - f[3]) + (f[5] - f[6]) + (f[8] - f[7]);
  const R jy = (f[2] - f[4]) + (f[5] + f[6]) - (f[7] + f[8]);
  const R Fb = k.gb * th;  // buoyancy, along +y
  R ux, uy, Fx = R(0), Fy = Fb;
  if constexpr (MODEL == kSolidDarcy) {
    // rho0 u = j + (Fb - A rho0 u)/2, A = C (1 - fl)^2 / (fl^3 + eps): with
    // D = fl^3 + eps + C (1 - fl)^2 / 2, u = (fl^3 + eps)/D (j + Fb/2)/rho0
    // and the drag -A rho0 u = -C (1 - fl)^2 / D (j + Fb/2)
    const R ml = R(1) - fl;
    const R fl3e = fl * fl * fl + k.darcy_eps;
    const R cm = k.darcy_c * ml * ml;
    const R rD = R(1) / (fl3e + R(0.5) * cm);
    const R qy = jy + R(0.5) * Fb;
    const R s = fl3e * rD * k.inv_rho0;
    ux = s * jx;
    uy = s * qy;
    Fx = -(cm * rD) * jx;
    Fy = Fb - (cm * rD) * qy;
  } else {
    // velocity scaled by the liquid fraction, or free (bounce-back model)
    const R s = MODEL == kSolidPbb ? R(1) : fl;
    ux = s * jx * k.inv_rho0;
    uy = s * (jy + R(0.5) * Fb) * k.inv_rho0;
  }
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
    // the force has an x part only under the drag
    constexpr bool fx = MODEL == kSolidDarcy;
    const R a1x = fx ? k.dk1f * m1x - k.hk1f * Fx : k.dk1f * m1x;
    const R a1y = k.dk1f * m1y - k.hk1f * Fy;
    const R a2xx = fx ? k.dk2f * m2xx - k.hk2f * (R(2) * ux * Fx) : k.dk2f * m2xx;
    const R a2xy = k.dk2f * m2xy - k.hk2f * (fx ? ux * Fy + uy * Fx : ux * Fy);
    const R a2yy = k.dk2f * m2yy - k.hk2f * (R(2) * uy * Fy);
    const R uu15 = R(1.5) * (ux * ux + uy * uy);
    const R feq0 = w0 * (drho - k.rho0 * uu15);
    const R qa0 = -(a2xx + a2yy) * third;
    const PairTerms<R> t(ux, uy, a1x, a1y, a2xx, a2xy, a2yy);
    if constexpr (MODEL == kSolidPbb) {
      const R ns = R(1) - fl;
      f[0] = (R(1) - ns) * (k.omk0f * f[0] + (k.k0f * feq0 - R(4.5) * w0 * qa0)) + ns * f[0];
#pragma unroll
      for (int p = 0; p < 4; ++p) {
        const R w = R(pair_w(p));
        const R E = w * (drho + k.rho0 * (R(4.5) * t.cu[p] * t.cu[p] - uu15));
        const R O = R(3) * w * k.rho0 * t.cu[p];
        relax_pair_pbb<R>(f[pair_plus(p)], f[pair_minus(p)], k.omk0f, k.k0f, E, O,
                          R(3) * w * t.c1[p], R(4.5) * w * t.qa[p], ns);
      }
    } else {
      f[0] = k.omk0f * f[0] + (k.k0f * feq0 - R(4.5) * w0 * qa0);
#pragma unroll
      for (int p = 0; p < 4; ++p) {
        const R w = R(pair_w(p));
        const R E = w * (drho + k.rho0 * (R(4.5) * t.cu[p] * t.cu[p] - uu15));
        const R O = R(3) * w * k.rho0 * t.cu[p];
        relax_pair<R>(f[pair_plus(p)], f[pair_minus(p)], k.omk0f, k.k0f, E, O, R(3) * w * t.c1[p],
                      R(4.5) * w * t.qa[p]);
      }
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
    {
      const R geq0 = dH - Cpth + w0 * Cpth;
      const R qa0 = -(a2xx + a2yy) * third;
      g[0] = k.omk0g * g[0] + (k.k0g * geq0 - R(4.5) * w0 * qa0);
    }
    const PairTerms<R> t(ux, uy, a1x, a1y, a2xx, a2xy, a2yy);
#pragma unroll
    for (int p = 0; p < 4; ++p) {
      const R w = R(pair_w(p));
      const R E = w * Cpth;
      const R O = R(3) * w * CpT * t.cu[p];
      relax_pair<R>(g[pair_plus(p)], g[pair_minus(p)], k.omk0g, k.k0g, E, O, R(3) * w * t.c1[p],
                    R(4.5) * w * t.qa[p]);
    }
  }
}

// Blocked structure-of-arrays: each row is cut into 64-cell chunks (one
// wavefront), and a chunk stores its 18 population planes one after another,
// 64 values each.  A wavefront's 18 loads then fall in one contiguous 18 x 64
// run of memory instead of 18 distant planes, which DRAM pages and the
// Infinity Cache serve better; population k of a cell sits k * 64 elements
// after its base (CavDev::plane = 64).
__device__ __forceinline__ int64_t cell_base(const CavDev &c, int x, int y) {
  return ((int64_t)y * (c.pitch >> 6) + (x >> 6)) * (kPlanes * kWave) + (x & (kWave - 1));
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
    n.idx[i] = cell_base(c, nx_, ny_);
  }
}

__device__ __forceinline__ bool heated(const CavDev &c, int x, int y) {
  return y == 0 && x >= c.hlo && x <= c.hhi;
}

// Population access.  NT selects non-temporal loads and stores, which
// stream through the caches without keeping the lines (the right choice once
// a lattice is far larger than the last-level cache).
template <bool NT, typename S>
__device__ __forceinline__ S ld(const S *p) {
  if constexpr (NT)
    return __builtin_nontemporal_load(p);
  else
    return *p;
}
template <bool NT, typename S>
__device__ __forceinline__ void st(S *p, S v) {
  if constexpr (NT)
    __builtin_nontemporal_store(v, p);
  else
    *p = v;
}

// Natural pre-collision populations of a cell (state of A-A parity 0, or of
// the current lattice of the two-lattice pattern).
template <typename S, typename R, bool NT = false>
__device__ __forceinline__ void load_natural(const S *__restrict__ P, int64_t plane, int64_t idx,
                                             R (&f)[kQ], R (&g)[kQ]) {
#pragma unroll
  for (int i = 0; i < kQ; ++i) {
    f[i] = R(ld<NT>(P + i * plane + idx));
    g[i] = R(ld<NT>(P + (kQ + i) * plane + idx));
  }
}

// Pre-collision populations gathered from the neighbours' swapped slots
// (A-A parity 1); links from outside come back from the cell's own slot.
template <typename S, typename R, bool NT = false>
__device__ __forceinline__ void load_gather(const CavDev &c, const Coef<R> &k,
                                            const S *__restrict__ P, int x, int y, int64_t idx,
                                            R (&f)[kQ], R (&g)[kQ]) {
  Nbr n;
  neighbours(c, x, y, -1, n);
  const bool bottom_hot = !c.periodic_y && heated(c, x, y);
#pragma unroll
  for (int i = 0; i < kQ; ++i) {
    const int64_t src = n.in[i] ? opp(i) * c.plane + n.idx[i] : i * c.plane + idx;
    f[i] = R(ld<NT>(P + src));
    R v = R(ld<NT>(P + kQ * c.plane + src));
    if (cy(i) == 1 && bottom_hot && !n.in[i]) v = k.anti(i) - v;
    g[i] = v;
  }
}

// Post-collision populations scattered to the neighbours' natural slots;
// links leaving the cavity are reflected into the cell's opposite slot.
template <typename S, typename R, bool NT = false>
__device__ __forceinline__ void store_scatter(const CavDev &c, const Coef<R> &k,
                                              S *__restrict__ P, int x, int y, int64_t idx,
                                              const R (&f)[kQ], const R (&g)[kQ]) {
  Nbr n;
  neighbours(c, x, y, +1, n);
  const bool bottom_hot = !c.periodic_y && heated(c, x, y);
#pragma unroll
  for (int i = 0; i < kQ; ++i) {
    const int64_t dst = n.in[i] ? i * c.plane + n.idx[i] : opp(i) * c.plane + idx;
    st<NT>(P + dst, S(f[i]));
    R v = g[i];
    if (cy(i) == -1 && bottom_hot && !n.in[i]) v = k.anti(i) - v;
    st<NT>(P + kQ * c.plane + dst, S(v));
  }
}

template <typename S, typename R, bool NT = false>
__device__ __forceinline__ void store_swapped(S *__restrict__ P, int64_t plane, int64_t idx,
                                              const R (&f)[kQ], const R (&g)[kQ]) {
#pragma unroll
  for (int i = 0; i < kQ; ++i) {
    st<NT>(P + opp(i) * plane + idx, S(f[i]));
    st<NT>(P + (kQ + opp(i)) * plane + idx, S(g[i]));
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
template <typename S, typename R, int MODEL, bool NT = false>
__device__ __forceinline__ void update_cell(const CavDev &c, const Coef<R> &k, int mode, int x,
                                            int y) {
  const int64_t idx = cell_base(c, x, y);
  R f[kQ], g[kQ];
  if (mode == 0) {
    S *P = static_cast<S *>(c.pop[0]);
    load_natural<S, R, NT>(P, c.plane, idx, f, g);
    collide<R, MODEL>(k, f, g);
    store_swapped<S, R, NT>(P, c.plane, idx, f, g);
  } else if (mode == 1) {
    S *P = static_cast<S *>(c.pop[0]);
    load_gather<S, R, NT>(c, k, P, x, y, idx, f, g);
    collide<R, MODEL>(k, f, g);
    store_scatter<S, R, NT>(c, k, P, x, y, idx, f, g);
  } else {
    const S *A = static_cast<const S *>(c.parity ? c.pop[1] : c.pop[0]);
    S *B = static_cast<S *>(c.parity ? c.pop[0] : c.pop[1]);
    load_natural<S, R, NT>(A, c.plane, idx, f, g);
    collide<R, MODEL>(k, f, g);
    store_scatter<S, R, NT>(c, k, B, x, y, idx, f, g);
  }
  if (!c.periodic_y && heated(c, x, y)) add_strip_flux<R>(c, k, x, g);
}

// Calls fn(std::integral_constant<int, MODEL>) for the cavity's solid model.
template <typename Fn>
__host__ __device__ inline auto with_model(int model, Fn &&fn) {
  switch (model) {
    case kSolidDarcy: return fn(std::integral_constant<int, kSolidDarcy>{});
    case kSolidPbb: return fn(std::integral_constant<int, kSolidPbb>{});
    default: return fn(std::integral_constant<int, kSolidScale>{});
  }
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

// Tile handled by workgroup b of nb: XCD bands or plain order, optionally
// walked backwards.  Alternating the walk direction between steps makes a step
// start where the previous one ended, on the lines the last-level cache holds.
__device__ __forceinline__ int tile_of(int b, int nb, bool bands, bool backwards) {
  if (!bands) return backwards ? nb - 1 - b : b;
  const int xcd = b % kXcds, local = b / kXcds;
  const int q = nb / kXcds, r = nb % kXcds;
  const int count = q + (xcd < r ? 1 : 0);
  const int start = xcd < r ? xcd * (q + 1) : r * (q + 1) + (xcd - r) * q;
  return start + (backwards ? count - 1 - local : local);
}

}  // namespace dev
}  // namespace lbm
