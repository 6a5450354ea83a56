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

// The rates of a cavity in the arithmetic type R of the update, read from
// its descriptor (computed on the host, Rates).  They are wavefront-uniform
// and land in scalar registers.  VREG = true moves each into a vector
// register instead: the fused kernels, whose walks hold many scalars of their
// own, would otherwise spill the rates to vector-register lanes and read
// them back with an instruction per use.
template <typename R, bool VREG = false>
struct Coef : Rates<R> {
  __device__ explicit Coef(const CavDev &c) : Rates<R>(rates_of(c)) {
    if constexpr (VREG) {
      static_assert(sizeof(Rates<R>) % sizeof(R) == 0, "rates are an array of R");
      R *p = reinterpret_cast<R *>(static_cast<Rates<R> *>(this));
#pragma unroll
      for (int i = 0; i < (int)(sizeof(Rates<R>) / sizeof(R)); ++i) p[i] = in_vgpr(p[i]);
    }
  }

 private:
  __device__ static const Rates<R> &rates_of(const CavDev &c) {
    if constexpr (sizeof(R) == 8)
      return c.r64;
    else
      return c.r32;
  }
  // a copy of a uniform value in a vector register (removed if unused)
  __device__ static R in_vgpr(R x) {
    R y;
    if constexpr (sizeof(R) == 8)
      asm("v_mov_b64 %0, %1" : "=v"(y) : "s"(x));
    else
      asm("v_mov_b32 %0, %1" : "=v"(y) : "s"(x));
    return y;
  }
};

template <typename R>
__device__ __forceinline__ R sel(bool p, R a, R b) {
  return p ? a : b;
}

// Sec. 2 below Eq. (1): H = Cp T + fl L with isothermal melting at Tm, in
// shifted form dH = H - Cp Tm, theta = T - Tm.  The latent part of the
// enthalpy is dH clamped to [0, L]: fl is that part over L, and theta is what
// lies outside it over Cp (exactly 0 in the mushy range).
template <typename R>
__device__ __forceinline__ void enthalpy_map(R dH, R L, R inv_L, R inv_Cp, R &fl, R &th) {
  const R lat = fmin(fmax(dH, R(0)), L);
  fl = fmin(fmax(dH * inv_L, R(0)), R(1));
  th = (dH - lat) * inv_Cp;
}

// Zeroth, first and second moments of nine populations, with the partial
// sums of opposite pairs shared between them.
template <typename R>
struct Moments {
  R m0, jx, jy, pxx, pyy, pxy;
  __device__ explicit Moments(const R (&p)[kQ]) {
    const R s13 = p[1] + p[3], d13 = p[1] - p[3];
    const R s24 = p[2] + p[4], d24 = p[2] - p[4];
    const R s56 = p[5] + p[6], d56 = p[5] - p[6];
    const R s78 = p[7] + p[8], d87 = p[8] - p[7];
    const R diag = s56 + s78;
    m0 = (p[0] + s13) + (s24 + diag);
    jx = d13 + (d56 + d87);
    jy = d24 + (s56 - s78);
    pxx = s13 + diag;
    pyy = s24 + diag;
    pxy = d56 - d87;
  }
};

// Relaxation of Eq. (2) in pair form.  With the combined first- and
// second-moment corrections a1, a2, Eq. (2) reads
//   p_i* = (1 - k0) p_i + k0 peq_i - 3 w_i c_i.a1 - (9/2) w_i Q_i:a2,
// Q_i = c_i c_i - I/3.  Under c -> -c the terms split into a part E that
// is even (the even equilibrium part and the Q:a2 term) and a part O that is
// odd (the odd equilibrium part and the c.a1 term), so the two members of an
// opposite pair (i, opp(i)) are
//   p_{+/-}* = (1 - k0) p_{+/-} + (E +/- O).
// The four pairs, "+" member first: (1, 3) along x, (2, 4) along y, (5, 7)
// along (1, 1), (6, 8) along (-1, 1); w = 1/9 on the axes, 1/36 on the
// diagonals.  With the second-moment corrections given as a2/6, the Q:a2
// parts of E, -(9/2) w Q_i:a2, are
//   axis x: -(1/2)(2/3 a2xx - 1/3 a2yy) = -2 (a2xx/6) + a2yy/6, axis y alike;
//   diagonals: -(1/8)(2/3 (a2xx + a2yy) +/- 2 a2xy)
//            = -(1/2)(a2xx/6 + a2yy/6) -/+ (3/2)(a2xy/6);
// and with v/3 = (k0 (first moment of the equilibrium) - a1)/3 the O parts,
// 3 w c_i.v, are v_x/3, v_y/3 on the axes and (+/-v_x/3 + v_y/3)/4 on the
// diagonals.  Each pair is relaxed as soon as its two terms exist, so few
// temporaries are live at once.
// With k0 = 1 (UNIT) the (1 - k0) p term is dropped.
template <typename R, bool UNIT>
__device__ __forceinline__ void relax_pair(R &pp, R &pm, R omk0, R E, R O) {
  if constexpr (UNIT) {
    pp = E + O;
    pm = E - O;
  } else {
    pp = omk0 * pp + (E + O);
    pm = omk0 * pm + (E - O);
  }
}

// One B-TriRT collision of a cell, shifted populations in place.  MODEL is
// the kernel variant: the solid-phase treatment of the flow (kSolid*), or
// kScaleUnitK0 (the scaled-velocity treatment with k0 = 1 for f and g),
// fixed at compile time.
template <typename R, int MODEL>
__device__ __forceinline__ void collide(const Rates<R> &k, R (&f)[kQ], R (&g)[kQ]) {
  constexpr int SOLID = MODEL == kScaleUnitK0 ? kSolidScale : MODEL;
  constexpr bool UNIT = MODEL == kScaleUnitK0;
  constexpr R third = R(1.0 / 3.0);
  // (a) total enthalpy (the other moments of g are taken in (e), so that
  // they are not held through the flow part)
  const R dH = ((g[0] + g[1]) + (g[2] + g[3])) + ((g[4] + g[5]) + (g[6] + g[7])) + g[8];
  // (b) liquid fraction and Cp theta (the map of enthalpy_map: the latent part
  // is dH clamped to [0, L], and Cp theta is what lies outside it)
  const R lat = fmin(fmax(dH, R(0)), k.L);
  const R fl = fmin(fmax(dH * k.inv_L, R(0)), R(1));
  const R Cpth = dH - lat;
  // (c) flow moments, buoyancy, momentum rho0 u immobilised in the solid
  const Moments<R> mf(f);
  const R Fb = k.gbc * Cpth;  // buoyancy rho0 g beta theta, along +y
  R ux, uy, rux, ruy, Fx = R(0), Fy = Fb;
  if constexpr (SOLID == kSolidDarcy) {
    // rho0 u = j + (Fb - A rho0 u)/2, A = C (1 - fl)^2 / (fl^3 + eps): with
    // D = fl^3 + eps + C (1 - fl)^2 / 2, u = (fl^3 + eps)/D (j + Fb/2)/rho0
    // and the drag -A rho0 u = -C (1 - fl)^2 / D (j + Fb/2)
    const R ml = R(1) - fl;
    const R fl3e = fl * fl * fl + k.darcy_eps;
    const R cm = k.darcy_c * ml * ml;
    const R rD = R(1) / (fl3e + R(0.5) * cm);
    const R qy = mf.jy + R(0.5) * Fb;
    const R s = fl3e * rD * k.inv_rho0;
    ux = s * mf.jx;
    uy = s * qy;
    Fx = -(cm * rD) * mf.jx;
    Fy = Fb - (cm * rD) * qy;
    rux = k.rho0 * ux;
    ruy = k.rho0 * uy;
  } else {
    // rho0 u = j + F/2, scaled by the liquid fraction (or free: bounce-back model)
    const R qy = mf.jy + R(0.5) * Fb;
    rux = SOLID == kSolidPbb ? mf.jx : fl * mf.jx;
    ruy = SOLID == kSolidPbb ? qy : fl * qy;
    ux = k.inv_rho0 * rux;
    uy = k.inv_rho0 * ruy;
  }
  // (d) flow collision with the Hermite-projected force:
  //   a1 = (k1 - k0)(j - rho0 u) - (1 - k1/2) F,
  //   a2 = (k2 - k0)(Pi - rho0 u u - drho I/3) - (1 - k2/2)(u F + F u)
  // (Pi the second moment); the odd parts need k0 rho0 u - a1
  // = k1 rho0 u - (k1 - k0) j + (1 - k1/2) F.
  {
    constexpr bool fx = SOLID == kSolidDarcy;  // the force has an x part only under the drag
    const R rxx = rux * ux, ryy = ruy * uy;
    const R r3 = mf.m0 * third;
    const R hF = k.hk2f3 * Fy;
    const R a6xx = fx ? k.dk2f6 * (mf.pxx - (r3 + rxx)) - k.hk2f3 * (ux * Fx)
                      : k.dk2f6 * (mf.pxx - (r3 + rxx));
    const R a6yy = k.dk2f6 * (mf.pyy - (r3 + ryy)) - hF * uy;
    const R a6xy = k.dk2f6 * (mf.pxy - rux * uy) -
                   R(0.5) * (fx ? hF * ux + k.hk2f3 * (uy * Fx) : hF * ux);
    const R vx3 = fx ? (k.k1f3 * rux - k.dk1f3 * mf.jx) + k.hk1f3 * Fx : k.k1f3 * rux - k.dk1f3 * mf.jx;
    const R vy3 = (k.k1f3 * ruy - k.dk1f3 * mf.jy) + k.hk1f3 * Fy;
    // k0 w X with X = drho - (3/2) rho0 u.u is the equilibrium without its
    // c.u terms; k0 (9/2) w rho0 (c.u)^2 adds the rest of its even part
    const R b9 = k.k0f9 * (mf.m0 - R(1.5) * (rxx + ryy));
    const R tr6 = a6xx + a6yy;
    const R t36 = R(0.25) * b9 - R(0.5) * tr6;
    const R rcu2 = (rux + ruy) * (ux + uy), rcu3 = (ruy - rux) * (uy - ux);
    R pre[kQ];
    if constexpr (SOLID == kSolidPbb) {
#pragma unroll
      for (int i = 0; i < kQ; ++i) pre[i] = f[i];
    }
    relax_pair<R, UNIT>(f[1], f[3], k.omk0f, k.k0h * rxx + ((b9 - R(2) * a6xx) + a6yy), vx3);
    relax_pair<R, UNIT>(f[2], f[4], k.omk0f, k.k0h * ryy + ((b9 - R(2) * a6yy) + a6xx), vy3);
    relax_pair<R, UNIT>(f[5], f[7], k.omk0f, k.k0e * rcu2 + (t36 - R(1.5) * a6xy), R(0.25) * (vx3 + vy3));
    relax_pair<R, UNIT>(f[6], f[8], k.omk0f, k.k0e * rcu3 + (t36 + R(1.5) * a6xy), R(0.25) * (vy3 - vx3));
    // rest population: k0 w0 X - (9/2) w0 Q_0:a2 = 4 (k0 X/9) + 4 (a2xx + a2yy)/6
    const R f0 = UNIT ? R(4) * (b9 + tr6) : k.omk0f * f[0] + R(4) * (b9 + tr6);
    if constexpr (SOLID == kSolidPbb) {
      // partial bounce-back: each member mixes its post-collision value with
      // its partner's pre-collision one, weighted by the solid fraction
      const R ns = R(1) - fl;
      f[0] = (R(1) - ns) * f0 + ns * pre[0];
#pragma unroll
      for (int i = 1; i < kQ; ++i) f[i] = (R(1) - ns) * f[i] + ns * pre[opp(i)];
    } else {
      f[0] = f0;
    }
  }
  // (e) enthalpy collision with the equilibrium of Eq. (3):
  //   geq_0 = dH - (1 - w0) Cp theta, geq_i = w_i (Cp theta + 3 Cp T c_i.u);
  //   a1 = (k1 - k0)(q - Cp T u), a2 = (k2 - k0)(Pi - Cp theta I/3)
  // (q, Pi the first and second moments of g); the odd parts need
  // k0 Cp T u - a1 = k1 Cp T u - (k1 - k0) q.
  {
    const Moments<R> mg(g);
    const R c3 = Cpth * third;
    const R a6xx = k.dk2g6 * (mg.pxx - c3);
    const R a6yy = k.dk2g6 * (mg.pyy - c3);
    const R a6xy = k.dk2g6 * mg.pxy;
    const R kT = k.k1g3 * (k.CpTm + Cpth);
    const R vx3 = kT * ux - k.dk1g3 * mg.jx;
    const R vy3 = kT * uy - k.dk1g3 * mg.jy;
    const R b9 = k.k0g9 * Cpth;
    const R tr6 = a6xx + a6yy;
    const R t36 = R(0.25) * b9 - R(0.5) * tr6;
    // rest population: k0 (dH - (5/9) Cp theta) + 4 (a2xx + a2yy)/6
    const R g0 = UNIT ? (k.k0g * dH - R(5) * b9) + R(4) * tr6
                     : k.omk0g * g[0] + ((k.k0g * dH - R(5) * b9) + R(4) * tr6);
    relax_pair<R, UNIT>(g[1], g[3], k.omk0g, (b9 - R(2) * a6xx) + a6yy, vx3);
    relax_pair<R, UNIT>(g[2], g[4], k.omk0g, (b9 - R(2) * a6yy) + a6xx, vy3);
    relax_pair<R, UNIT>(g[5], g[7], k.omk0g, t36 - R(1.5) * a6xy, R(0.25) * (vx3 + vy3));
    relax_pair<R, UNIT>(g[6], g[8], k.omk0g, t36 + R(1.5) * a6xy, R(0.25) * (vy3 - vx3));
    g[0] = g0;
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
__device__ __forceinline__ void load_gather(const CavDev &c, const Rates<R> &k,
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
__device__ __forceinline__ void store_scatter(const CavDev &c, const Rates<R> &k,
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
__device__ __forceinline__ void add_strip_flux(const CavDev &c, const Rates<R> &k, int x,
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
__device__ __forceinline__ void update_cell(const CavDev &c, const Rates<R> &k, int mode, int x,
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

// The same for a kernel variant (CavDev::kmodel), kScaleUnitK0 included.
template <typename Fn>
__host__ __device__ inline auto with_kernel_model(int kmodel, Fn &&fn) {
  if (kmodel == kScaleUnitK0) return fn(std::integral_constant<int, kScaleUnitK0>{});
  return with_model(kmodel, static_cast<Fn &&>(fn));
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
