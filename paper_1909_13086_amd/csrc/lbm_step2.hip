// Two or three time steps per launch for the two-lattice pattern (temporal
// blocking).  The two-step kernel is described here; the three-step kernel,
// which extends it by one level, further below.
//
// One launch reads the natural state at time t from lattice A once and writes
// the natural state at t+2 to lattice B once, so a pair of steps moves the
// bytes of one.  Each wavefront owns a strip of 62 columns and a segment of
// `seg` rows and walks along the segment with a three-row window in
// registers:
//   - first step (a collision of the loaded state) for the segment's rows and
//     one halo row on each side, columns x0-1 .. x0+62 (the halo cells are
//     recomputed by the neighbouring wavefronts as well);
//   - second step for the owned cells: the streamed populations are taken
//     from the window (from the neighbouring lane for x shifts, a wavefront
//     shuffle), walls reflect into the cell's own first-step values exactly as
//     the single-step kernels do, the collision runs again and the result is
//     scattered to B.
// Every collision is the same code as in the single-step kernels, so a launch
// equals two single two-lattice steps bit for bit.
//
// Rows reach the registers in one of two ways:
//   - direct: each row is loaded from A when the walk needs it;
//   - staged: rows are copied from A into a per-wavefront LDS double buffer by
//     asynchronous global-to-LDS loads issued one row ahead, so the fetch of
//     the next row overlaps the two collisions of the current one without
//     holding registers.
#include "lbm_device.h"

#include <utility>

namespace lbm {
namespace {

using namespace dev;

constexpr int kDirectWaves = 4;        // wavefronts per workgroup, direct rows
constexpr int kStagedWaves = 2;        // wavefronts per workgroup, staged rows
// wavefronts per workgroup of the single-cavity three-step launch: one, so a
// CU starts a new segment as soon as any wavefront finishes (its 18 KiB of LDS
// are its own)
constexpr int kStep3Waves = 1;

// The three populations that move along the walk direction D (c_y = D):
// 2, 5, 6 going up, 4, 7, 8 going down -> window slots 0, 1, 2.
template <int D>
__device__ constexpr int along_slot(int i) {
  return D > 0 ? (i == 2 ? 0 : (i == 5 ? 1 : 2)) : (i == 4 ? 0 : (i == 7 ? 1 : 2));
}

// Wavefront-wide lane shifts by one lane (DPP wave_shr:1 / wave_shl:1): a
// lane receives the value of lane - 1 or lane + 1; the first or last lane,
// which has no source, keeps its own value.
constexpr int kDppWaveShr1 = 0x138;
constexpr int kDppWaveShl1 = 0x130;

template <int CTRL>
__device__ __forceinline__ float dpp_shift(float v) {
  const int i = __float_as_int(v);
  return __int_as_float(__builtin_amdgcn_update_dpp(i, i, CTRL, 0xf, 0xf, false));
}
template <int CTRL>
__device__ __forceinline__ double dpp_shift(double v) {
  const int lo = __double2loint(v), hi = __double2hiint(v);
  return __hiloint2double(__builtin_amdgcn_update_dpp(hi, hi, CTRL, 0xf, 0xf, false),
                          __builtin_amdgcn_update_dpp(lo, lo, CTRL, 0xf, 0xf, false));
}

template <typename R>
__device__ __forceinline__ R lane_from(R v, int dx) {
  // value of the lane holding column x - dx
  if (dx > 0) return dpp_shift<kDppWaveShr1>(v);
  if (dx < 0) return dpp_shift<kDppWaveShl1>(v);
  return v;
}

// Column of one lane of a strip.
struct Col {
  int x, xw;          // column (-H .. nx+H-1) and its periodic wrap
  bool real;          // the column exists (owners, and halo columns that wrap)
  bool owner;         // lanes 1 .. 62 inside the cavity
  bool bottom_hot;    // heated column of a non-periodic bottom wall
  bool strip_flux;    // counts the first-step strip flux of row 0
};

// Halo columns and rows lie at most H cells outside the cavity (H = 1 for
// two steps per launch, 2 for three).  With periodic sides they wrap, at
// most H times for a cavity narrower than H.
template <int H>
__device__ __forceinline__ int wrap_near(int v, int n) {
#pragma unroll
  for (int i = 0; i < H; ++i) v = v < 0 ? v + n : (v >= n ? v - n : v);
  return v;
}
template <int H = 1>
__device__ __forceinline__ bool col_real(const CavDev &c, int x) {
  return (x >= 0 && x < c.nx) || (c.periodic_x && x >= -H && x < c.nx + H);
}
template <int H = 1>
__device__ __forceinline__ int col_wrap(const CavDev &c, int x) {
  return wrap_near<H>(x, c.nx);
}
template <int H = 1>
__device__ __forceinline__ bool row_real(const CavDev &c, int r) {
  return (r >= 0 && r < c.ny) || (c.periodic_y && r >= -H && r < c.ny + H);
}
template <int H = 1>
__device__ __forceinline__ int row_wrap(const CavDev &c, int r) {
  return wrap_near<H>(r, c.ny);
}

// H: halo columns on each side of the strip (one per step after the first)
template <int H = 1>
__device__ __forceinline__ Col make_col(const CavDev &c, int x, int lane, int y0) {
  Col q;
  q.x = x;
  q.real = col_real<H>(c, x);
  q.xw = col_wrap<H>(c, x);
  q.owner = lane >= H && lane < kWave - H && x < c.nx;
  // a halo column across a periodic side is heated as the column it wraps to
  q.bottom_hot = !c.periodic_y && q.xw >= c.hlo && q.xw <= c.hhi;
  // the segment that owns row 0 computes that row's first step exactly once
  q.strip_flux = q.owner && q.bottom_hot && y0 == 0;
  return q;
}

// First step of a loaded row: collision, plus the strip flux of a heated
// bottom cell's first step.
template <typename R, int MODEL>
__device__ __forceinline__ void first_collide(const CavDev &c, const Rates<R> &k, const Col &q, int r,
                                              R (&f)[kQ], R (&g)[kQ]) {
  collide<R, MODEL>(k, f, g);
  if (r == 0 && q.strip_flux) add_strip_flux<R>(c, k, q.x, g);
}

template <typename R>
__device__ __forceinline__ void zero_row(R (&f)[kQ], R (&g)[kQ]) {
#pragma unroll
  for (int i = 0; i < kQ; ++i) f[i] = g[i] = R(0);
}

// Second step of row y: the streamed state gathered from the window, walls
// applied (WALLS = false: the wavefront's cells and their neighbours are all
// inside the cavity, no link crosses a wall), then collided (result in pf,
// pg).
template <typename R, int D, bool WALLS, int MODEL>
__device__ __forceinline__ void second_collide(const CavDev &c, const Rates<R> &k, const Col &q, int y,
                                               const R (&cf)[kQ], const R (&cg)[kQ],
                                               const R (&nf)[kQ], const R (&ng)[kQ],
                                               const R (&af)[3], const R (&ag)[3], R (&pf)[kQ],
                                               R (&pg)[kQ]) {
  const bool xm_in = c.periodic_x || q.x - 1 >= 0;
  const bool xp_in = c.periodic_x || q.x + 1 < c.nx;
  const bool ym_in = c.periodic_y || y - 1 >= 0;
  const bool yp_in = c.periodic_y || y + 1 < c.ny;
  const bool hot = q.bottom_hot && y == 0;
#pragma unroll
  for (int i = 0; i < kQ; ++i) {
    const int ex = cx(i), ey = cy(i);
    R vf, vg;
    if (ey == 0) {
      vf = cf[i];
      vg = cg[i];
    } else if (ey == D) {
      vf = af[along_slot<D>(i)];
      vg = ag[along_slot<D>(i)];
    } else {
      vf = nf[i];
      vg = ng[i];
    }
    vf = lane_from(vf, ex);
    vg = lane_from(vg, ex);
    const bool in_x = ex > 0 ? xm_in : (ex < 0 ? xp_in : true);
    const bool in_y = ey > 0 ? ym_in : (ey < 0 ? yp_in : true);
    if (WALLS && !(in_x && in_y)) {
      // the link crossed a wall: it comes back from the cell itself
      vf = cf[opp(i)];
      vg = cg[opp(i)];
      if (ey == 1 && hot) vg = k.anti(i) - vg;
    }
    pf[i] = vf;
    pg[i] = vg;
  }
  collide<R, MODEL>(k, pf, pg);
}

// The same for the third step of the ring walk: row y's own populations are
// read from its LDS ring slot where they are used (the centre populations,
// and the reflected ones of links that crossed a wall), instead of being held
// in registers.  slot points at this lane's value of population 0.
template <typename R, int D, bool WALLS, int MODEL>
__device__ __forceinline__ void third_collide(const CavDev &c, const Rates<R> &k, const Col &q, int y,
                                              const R *slot, const R (&nf)[kQ], const R (&ng)[kQ],
                                              const R (&af)[3], const R (&ag)[3], R (&pf)[kQ],
                                              R (&pg)[kQ]) {
  const bool xm_in = c.periodic_x || q.x - 1 >= 0;
  const bool xp_in = c.periodic_x || q.x + 1 < c.nx;
  const bool ym_in = c.periodic_y || y - 1 >= 0;
  const bool yp_in = c.periodic_y || y + 1 < c.ny;
  const bool hot = q.bottom_hot && y == 0;
#pragma unroll
  for (int i = 0; i < kQ; ++i) {
    const int ex = cx(i), ey = cy(i);
    R vf, vg;
    if (ey == 0) {
      vf = slot[i * kWave];
      vg = slot[(kQ + i) * kWave];
    } else if (ey == D) {
      vf = af[along_slot<D>(i)];
      vg = ag[along_slot<D>(i)];
    } else {
      vf = nf[i];
      vg = ng[i];
    }
    vf = lane_from(vf, ex);
    vg = lane_from(vg, ex);
    const bool in_x = ex > 0 ? xm_in : (ex < 0 ? xp_in : true);
    const bool in_y = ey > 0 ? ym_in : (ey < 0 ? yp_in : true);
    if (WALLS && !(in_x && in_y)) {
      // the link crossed a wall: it comes back from the cell itself
      vf = slot[opp(i) * kWave];
      vg = slot[(kQ + opp(i)) * kWave];
      if (ey == 1 && hot) vg = k.anti(i) - vg;
    }
    pf[i] = vf;
    pg[i] = vg;
  }
  collide<R, MODEL>(k, pf, pg);
}

// Post-collision populations of an interior cell pushed to its neighbours'
// natural slots: three row bases (wavefront-uniform) and three column
// offsets within a row, so every address is a row pointer plus a 32-bit
// offset.
template <typename S, typename R>
__device__ __forceinline__ void store_interior(const CavDev &c, S *__restrict__ B, int x, int y,
                                               const R (&f)[kQ], const R (&g)[kQ]) {
  const int64_t row_elems = (int64_t)(c.pitch >> 6) * (kPlanes * kWave);
  S *rows[3];
  uint32_t cols[3];
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    rows[d] = B + (int64_t)(y - 1 + d) * row_elems;
    const int xx = x - 1 + d;
    cols[d] = (uint32_t)((xx >> 6) * (kPlanes * kWave) + (xx & (kWave - 1)));
  }
#pragma unroll
  for (int i = 0; i < kQ; ++i) {
    S *r = rows[cy(i) + 1];
    const uint32_t o = cols[cx(i) + 1] + (uint32_t)(i * kWave);
    r[o] = S(f[i]);
    r[o + kQ * kWave] = S(g[i]);
  }
}

// Stores of an owned cell's second step (and its strip flux).
// FLUX = false: the strip flux of this step was already counted.
template <typename S, typename R, bool WALLS = true, bool FLUX = true>
__device__ __forceinline__ void emit(const CavDev &c, const Rates<R> &k, S *__restrict__ B, const Col &q,
                                     int y, const R (&pf)[kQ], const R (&pg)[kQ]) {
  if (q.owner) {
    if constexpr (WALLS) {
      store_scatter<S, R>(c, k, B, q.x, y, cell_base(c, q.x, y), pf, pg);
      if (FLUX && q.bottom_hot && y == 0) add_strip_flux<R>(c, k, q.x, pg);
    } else {
      store_interior<S, R>(c, B, q.x, y, pf, pg);
    }
  }
}

// No cell within H cells of the strip segment [x0, x0 + 64 - 2H) x [y0, y1)
// lies on or beyond a wall or a periodic seam, so no link of a cell whose
// collision feeds an owned cell crosses one.
template <int H = 1>
__device__ __forceinline__ bool interior_segment(const CavDev &c, int x0, int y0, int y1) {
  return x0 >= H && x0 + (kWave - 2 * H) + H <= c.nx && y0 >= H && y1 + H <= c.ny;
}

// Window slide: (a, c) <- (populations of c moving along D, n).
template <int D, typename R>
__device__ __forceinline__ void slide(R (&af)[3], R (&ag)[3], R (&cf)[kQ], R (&cg)[kQ],
                                      const R (&nf)[kQ], const R (&ng)[kQ]) {
  constexpr int a0 = D > 0 ? 2 : 4, a1 = D > 0 ? 5 : 7, a2 = D > 0 ? 6 : 8;
  af[0] = cf[a0]; af[1] = cf[a1]; af[2] = cf[a2];
  ag[0] = cg[a0]; ag[1] = cg[a1]; ag[2] = cg[a2];
#pragma unroll
  for (int i = 0; i < kQ; ++i) {
    cf[i] = nf[i];
    cg[i] = ng[i];
  }
}

// Rows y0 .. y1-1 of one strip, walked in direction D (+1 upwards from y0,
// -1 downwards from y1-1), each row loaded from A when needed.  Adjacent
// segments walking in opposite directions reach the two halo rows they share
// at the same point of their walks, so the second reader finds them in L2.
template <typename S, typename R, int D, int MODEL>
__device__ __forceinline__ void walk_direct(const CavDev &c, const Rates<R> &k, const S *__restrict__ A,
                                            S *__restrict__ B, const Col &q, int y0, int y1) {
  auto first_step = [&](int r, R (&f)[kQ], R (&g)[kQ]) {
    // zeros when the row or column does not exist; such values are never used
    if (!(row_real(c, r) && q.real)) {
      zero_row(f, g);
      return;
    }
    load_natural<S, R>(A, c.plane, cell_base(c, q.xw, row_wrap(c, r)), f, g);
    first_collide<R, MODEL>(c, k, q, r, f, g);
  };
  const int ys = D > 0 ? y0 : y1 - 1;
  const int ye = D > 0 ? y1 : y0 - 1;
  R cf[kQ], cg[kQ];      // first-step state of row y
  R nf[kQ], ng[kQ];      // first-step state of row y + D
  R af[3], ag[3];        // populations of row y - D moving along the walk
  first_step(ys - D, cf, cg);
  first_step(ys, nf, ng);
  slide<D>(af, ag, cf, cg, nf, ng);
  for (int y = ys; y != ye; y += D) {
    first_step(y + D, nf, ng);
    R pf[kQ], pg[kQ];
    second_collide<R, D, true, MODEL>(c, k, q, y, cf, cg, nf, ng, af, ag, pf, pg);
    emit<S, R>(c, k, B, q, y, pf, pg);
    slide<D>(af, ag, cf, cg, nf, ng);
  }
}

// ---- staged rows --------------------------------------------------------

// s_waitcnt immediates (vmcnt in bits 3:0 and 15:14, expcnt 6:4, lgkmcnt 11:8)
constexpr int kWaitVm0 = 0x0F70;    // vector memory count 0, others unconstrained
constexpr int kWaitLgkm0 = 0xC07F;  // LDS/scalar count 0, others unconstrained

__device__ __forceinline__ void wait_vm() {
  asm volatile("" ::: "memory");
  __builtin_amdgcn_s_waitcnt(kWaitVm0);
  asm volatile("" ::: "memory");
}
__device__ __forceinline__ void wait_lgkm() {
  asm volatile("" ::: "memory");
  __builtin_amdgcn_s_waitcnt(kWaitLgkm0);
  asm volatile("" ::: "memory");
}

template <typename T>
__device__ __forceinline__ __attribute__((address_space(3))) void *lds_addr(T *p) {
  return (__attribute__((address_space(3))) void *)p;
}

// Global-to-LDS copy lanes of a strip row.  The copy moves 4 bytes per lane
// and instruction and writes lane l's bytes at LDS offset 4 l: FP32 rows take
// one instruction per plane (lane l copies cell l), FP64 rows two (lanes 2m
// and 2m+1 copy the low and high words of cell m of each half row).  Lanes
// whose cell does not exist copy the row's first cell instead, so every copy
// stays inside the lattice; the lanes of such cells never read their slots.
struct CopyLanes {
  uint32_t off[2];  // byte offset of the copied word within the row
};

// xa: column of lane 0
template <typename S, int H = 1>
__device__ __forceinline__ CopyLanes copy_lanes(const CavDev &c, int xa, int lane) {
  CopyLanes L;
  const uint32_t sub = sizeof(S) == 8 ? 4u * (lane & 1) : 0u;
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    const int m = sizeof(S) == 8 ? h * (kWave / 2) + (lane >> 1) : lane;
    const int x = xa + m;
    const uint32_t e = col_real<H>(c, x) ? (uint32_t)cell_base(c, col_wrap<H>(c, x), 0) : 0u;
    L.off[h] = e * (uint32_t)sizeof(S) + sub;
  }
  return L;
}

// Copy of plane I of a row.  The instruction's immediate offset moves the
// global and the LDS address together; it is kept below 4096 bytes by
// stepping both bases once per group of planes.
template <typename S, int I>
__device__ __forceinline__ void copy_plane(const char *base, const CopyLanes &L, S *buf) {
  constexpr int plane_bytes = kWave * sizeof(S);
  constexpr int per_group = 4096 / plane_bytes;
  constexpr int group_bytes = per_group * plane_bytes;
  constexpr int grp = I / per_group, imm = (I % per_group) * plane_bytes;
  const char *g = base + grp * group_bytes;
  S *l = buf + grp * (group_bytes / (int)sizeof(S));
  if constexpr (sizeof(S) == 8) {
    __builtin_amdgcn_global_load_lds(g + L.off[0], lds_addr(l), 4, imm, 0);
    __builtin_amdgcn_global_load_lds(g + L.off[1], lds_addr(l + kWave / 2), 4, imm, 0);
  } else {
    __builtin_amdgcn_global_load_lds(g + L.off[0], lds_addr(l), 4, imm, 0);
  }
}

template <typename S, int... I>
__device__ __forceinline__ void copy_planes(const char *base, const CopyLanes &L, S *buf,
                                            std::integer_sequence<int, I...>) {
  (copy_plane<S, I>(base, L, buf), ...);
}

// Issue the copy of row r of A into an LDS buffer of kPlanes x kWave values.
template <typename S, int H = 1>
__device__ __forceinline__ void copy_row(const CavDev &c, const S *__restrict__ A, const CopyLanes &L,
                                         int r, S *buf) {
  const int64_t row = (int64_t)row_wrap<H>(c, r) * (c.pitch >> 6) * (kPlanes * kWave);
  const char *base = reinterpret_cast<const char *>(A + row);
  asm volatile("" ::: "memory");
  copy_planes<S>(base, L, buf, std::make_integer_sequence<int, kPlanes>{});
  asm volatile("" ::: "memory");
}

template <typename S, typename R>
__device__ __forceinline__ void read_row(const S *buf, int lane, R (&f)[kQ], R (&g)[kQ]) {
#pragma unroll
  for (int i = 0; i < kQ; ++i) {
    f[i] = R(buf[i * kWave + lane]);
    g[i] = R(buf[(kQ + i) * kWave + lane]);
  }
}

// The same walk with rows staged through LDS.  Rows along the walk are
// numbered k = 0 (ys - D), 1 (ys), 2, ...; row k lives in buffer k & 1.  The
// copy of row k + 1 is issued into the buffer that row k - 1 has left, before
// row k is read and collided; it is waited for before the stores of that
// iteration are issued, so the stores never delay a later wait.
template <typename S, typename R, int D, bool WALLS, int MODEL>
__device__ __forceinline__ void walk_staged(const CavDev &c, const Rates<R> &k, const S *__restrict__ A,
                                            S *__restrict__ B, const Col &q, int y0, int y1, int x0,
                                            S *bufs) {
  const int lane = threadIdx.x & (kWave - 1);
  const CopyLanes L = copy_lanes<S>(c, x0 - 1, lane);
  auto buf = [&](int b) { return bufs + b * (kPlanes * kWave); };
  auto issue = [&](int r, int b) {
    if (row_real(c, r)) copy_row<S>(c, A, L, r, buf(b));
  };
  auto first_step = [&](int r, int b, R (&f)[kQ], R (&g)[kQ]) {
    // zeros when the row or column does not exist; such values are never used
    if (!(row_real(c, r) && q.real)) {
      zero_row(f, g);
      return;
    }
    read_row<S, R>(buf(b), lane, f, g);
    first_collide<R, MODEL>(c, k, q, r, f, g);
  };

  const int ys = D > 0 ? y0 : y1 - 1;
  const int ye = D > 0 ? y1 : y0 - 1;
  R cf[kQ], cg[kQ];      // first-step state of row y
  R nf[kQ], ng[kQ];      // first-step state of row y + D
  R af[3], ag[3];        // populations of row y - D moving along the walk
  issue(ys - D, 0);
  issue(ys, 1);
  wait_vm();
  first_step(ys - D, 0, cf, cg);
  wait_lgkm();           // buffer 0 has been read before it is refilled
  issue(ys + D, 0);
  first_step(ys, 1, nf, ng);
  slide<D>(af, ag, cf, cg, nf, ng);
  wait_vm();
  int b = 0;
  for (int y = ys; y != ye; y += D, b ^= 1) {
    wait_lgkm();         // buffer b ^ 1 (row y) has been read
    if (y + D != ye) issue(y + 2 * D, b ^ 1);
    first_step(y + D, b, nf, ng);
    R pf[kQ], pg[kQ];
    second_collide<R, D, WALLS, MODEL>(c, k, q, y, cf, cg, nf, ng, af, ag, pf, pg);
    wait_vm();
    emit<S, R, WALLS>(c, k, B, q, y, pf, pg);
    slide<D>(af, ag, cf, cg, nf, ng);
  }
}

// order: bit 0 XCD bands, bit 1 tiles walked backwards on odd parity,
// bit 2 odd segments walked downwards
template <typename S, typename R, bool STAGED, int MODEL>
__global__ __launch_bounds__(STAGED ? kStagedWaves * kWave : kDirectWaves * kWave)
__attribute__((amdgpu_waves_per_eu(2))) void k_step2(
    CavDev c, int strips_x, int nseg, int seg_rows, int order) {
  constexpr int waves = STAGED ? kStagedWaves : kDirectWaves;
  __shared__ S lds[STAGED ? waves * 2 * kPlanes * kWave : 1];
  const int lane = threadIdx.x & (kWave - 1);
  const int wid = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
  const int b = tile_of(blockIdx.x, gridDim.x, order & 1, (order & 2) && (c.parity & 1));
  const int w = b * waves + wid;
  if (w >= strips_x * nseg) return;  // uniform per wavefront; no barriers follow
  const int strip = w % strips_x, seg = w / strips_x;
  const int x0 = strip * kStripCols;
  const int y0 = seg * seg_rows;
  const int y1 = min(y0 + seg_rows, c.ny);
  const Col q = make_col(c, x0 - 1 + lane, lane, y0);
  const Coef<R, true> k(c);
  const S *__restrict__ A = static_cast<const S *>(c.parity ? c.pop[1] : c.pop[0]);
  S *__restrict__ B = static_cast<S *>(c.parity ? c.pop[0] : c.pop[1]);
  const bool down = (order & 4) && (seg & 1);
  if constexpr (STAGED) {
    S *bufs = lds + wid * 2 * kPlanes * kWave;
    const bool inner = interior_segment(c, x0, y0, y1);
    if (down) {
      if (inner)
        walk_staged<S, R, -1, false, MODEL>(c, k, A, B, q, y0, y1, x0, bufs);
      else
        walk_staged<S, R, -1, true, MODEL>(c, k, A, B, q, y0, y1, x0, bufs);
    } else {
      if (inner)
        walk_staged<S, R, +1, false, MODEL>(c, k, A, B, q, y0, y1, x0, bufs);
      else
        walk_staged<S, R, +1, true, MODEL>(c, k, A, B, q, y0, y1, x0, bufs);
    }
  } else {
    if (down)
      walk_direct<S, R, -1, MODEL>(c, k, A, B, q, y0, y1);
    else
      walk_direct<S, R, +1, MODEL>(c, k, A, B, q, y0, y1);
  }
}

template <typename S, typename R, bool STAGED>
hipError_t dispatch(const CavDev &c, const LaunchCfg &cfg, hipStream_t s) {
  if (cfg.seg < 1 || cfg.seg > kMaxSegmentRows) return hipErrorInvalidValue;
  const int strips_x = (c.nx + kStripCols - 1) / kStripCols;
  const int nseg = (c.ny + cfg.seg - 1) / cfg.seg;
  const int waves = strips_x * nseg;
  const int per_block = STAGED ? kStagedWaves : kDirectWaves;
  const dim3 grid((waves + per_block - 1) / per_block);
  const int order = (cfg.xcd ? 1 : 0) | (cfg.reverse ? 2 : 0) | (cfg.zigzag ? 4 : 0);
  with_kernel_model(c.kmodel, [&](auto m) {
    hipLaunchKernelGGL((k_step2<S, R, STAGED, decltype(m)::value>), grid, dim3(per_block * kWave), 0,
                       s, c, strips_x, nseg, cfg.seg, order);
    return 0;
  });
  return hipGetLastError();
}

// ---- three steps per launch ---------------------------------------------
//
// The same scheme one level deeper: a wavefront owns 60 columns (lanes
// 2 .. 61) of `seg` rows and walks them with two windows.  Rows are loaded
// and collided once (level 1) for the rows y0-2 .. y1+1; the level-1 window
// feeds the second step (level 2) of rows y0-1 .. y1, whose window feeds the
// third step (level 3) of the owned rows, which is stored.  FP32 keeps both
// windows in registers and stages rows through LDS as above (walk3_staged);
// FP64, whose two windows would exceed the register file, keeps the level-2
// window in LDS and loads rows directly (walk3_ring).  Level 2 runs on every
// lane; only lanes 1 .. 62 hold correct values there, which is all level 3
// of the owned lanes reads.  Rows outside the cavity give values that no
// owned cell uses (their links are reflected at the wall).  Each level is the
// single-step update, so a launch equals three single two-lattice steps bit
// for bit.
//
// Iteration y of the walk (direction D) computes level 1 of row y+2D, level 2
// of row y+D and level 3 of row y, then slides both windows by one row.  With
// STEPS = 2 the walk stores level 2 of the owned rows instead (a batched
// launch whose cavity has two steps left); its strip flux is counted where
// level 2 is computed.
template <typename S, typename R, int D, bool WALLS, int MODEL, int STEPS = 3>
__device__ __forceinline__ void walk3_staged(const CavDev &c, const Rates<R> &k, const S *__restrict__ A,
                                             S *__restrict__ B, const Col &q, int y0, int y1, int x0,
                                             S *bufs) {
  const int lane = threadIdx.x & (kWave - 1);
  const CopyLanes L = copy_lanes<S, 2>(c, x0 - 2, lane);
  auto buf = [&](int b) { return bufs + b * (kPlanes * kWave); };
  auto issue = [&](int r, int b) {
    if (row_real<2>(c, r)) copy_row<S, 2>(c, A, L, r, buf(b));
  };
  auto level1 = [&](int r, int b, R (&f)[kQ], R (&g)[kQ]) {
    if (!(row_real<2>(c, r) && q.real)) {
      zero_row(f, g);
      return;
    }
    read_row<S, R>(buf(b), lane, f, g);
    first_collide<R, MODEL>(c, k, q, r, f, g);
  };
  // level 2 of row r into (f, g), with the strip flux of row 0 (the segment
  // that owns row 0 computes its level 2 exactly once)
  auto level2 = [&](int r, const R (&cf)[kQ], const R (&cg)[kQ], const R (&nf)[kQ],
                    const R (&ng)[kQ], const R (&af)[3], const R (&ag)[3], R (&f)[kQ], R (&g)[kQ]) {
    second_collide<R, D, WALLS, MODEL>(c, k, q, r, cf, cg, nf, ng, af, ag, f, g);
    if (r == 0 && q.strip_flux) add_strip_flux<R>(c, k, q.x, g);
  };

  const int ys = D > 0 ? y0 : y1 - 1;
  const int ye = D > 0 ? y1 : y0 - 1;
  R c1f[kQ], c1g[kQ], n1f[kQ], n1g[kQ], a1f[3], a1g[3];  // level-1 window
  R c2f[kQ], c2g[kQ], n2f[kQ], n2g[kQ], a2f[3], a2g[3];  // level-2 window
  // prologue: level 1 of rows ys-2D .. ys+D, level 2 of rows ys-D and ys
  issue(ys - 2 * D, 0);
  issue(ys - D, 1);
  wait_vm();
  level1(ys - 2 * D, 0, c1f, c1g);
  wait_lgkm();
  issue(ys, 0);
  level1(ys - D, 1, n1f, n1g);
  slide<D>(a1f, a1g, c1f, c1g, n1f, n1g);
  wait_vm();
  wait_lgkm();
  issue(ys + D, 1);
  level1(ys, 0, n1f, n1g);
  level2(ys - D, c1f, c1g, n1f, n1g, a1f, a1g, c2f, c2g);
  slide<D>(a1f, a1g, c1f, c1g, n1f, n1g);
  wait_vm();
  wait_lgkm();
  issue(ys + 2 * D, 0);
  level1(ys + D, 1, n1f, n1g);
  level2(ys, c1f, c1g, n1f, n1g, a1f, a1g, n2f, n2g);
  slide<D>(a2f, a2g, c2f, c2g, n2f, n2g);
  slide<D>(a1f, a1g, c1f, c1g, n1f, n1g);
  wait_vm();
  int b = 0;
  for (int y = ys; y != ye; y += D, b ^= 1) {
    // row y+2D is in buffer b; buffer b^1 (row y+D) has been read
    wait_lgkm();
    if (y + D != ye) issue(y + 3 * D, b ^ 1);
    level1(y + 2 * D, b, n1f, n1g);
    level2(y + D, c1f, c1g, n1f, n1g, a1f, a1g, n2f, n2g);
    if constexpr (STEPS == 3) {
      R pf[kQ], pg[kQ];
      second_collide<R, D, WALLS, MODEL>(c, k, q, y, c2f, c2g, n2f, n2g, a2f, a2g, pf, pg);
      wait_vm();
      emit<S, R, WALLS>(c, k, B, q, y, pf, pg);
    } else {
      wait_vm();
      emit<S, R, WALLS, false>(c, k, B, q, y, c2f, c2g);
    }
    slide<D>(a2f, a2g, c2f, c2g, n2f, n2g);
    slide<D>(a1f, a1g, c1f, c1g, n1f, n1g);
  }
}

// ---- four steps per launch (FP32) ----------------------------------------
//
// The three-step walk one level deeper, for FP32 only (its three register
// windows fit the register file; FP64's do not): a wavefront owns 58 columns
// (lanes 3 .. 60; three halo columns each side) and a segment of `seg` rows;
// iteration y of the walk computes level 1 of row y+3D (from the row staged
// in LDS), level 2 of row y+2D, level 3 of row y+D and level 4 of row y,
// which is stored.  Level m is correct on lanes m-1 .. 64-m, which is all
// level m+1 of the owned lanes reads.  Rows are staged through the LDS double
// buffer one row ahead, as in the other walks.  Each level is the single-step
// update, so a launch equals four single two-lattice steps bit for bit; the
// strip flux of row 0 is counted at every level by the segment that owns it.
template <typename S, typename R, int D, bool WALLS, int MODEL>
__device__ __forceinline__ void walk4_staged(const CavDev &c, const Rates<R> &k, const S *__restrict__ A,
                                             S *__restrict__ B, const Col &q, int y0, int y1, int x0,
                                             S *bufs) {
  static_assert(sizeof(R) == 4, "four steps per launch are FP32 only");
  const int lane = threadIdx.x & (kWave - 1);
  const CopyLanes L = copy_lanes<S, 3>(c, x0 - 3, lane);
  auto buf = [&](int b) { return bufs + b * (kPlanes * kWave); };
  auto issue = [&](int r, int b) {
    if (row_real<3>(c, r)) copy_row<S, 3>(c, A, L, r, buf(b));
  };
  auto level1 = [&](int r, int b, R (&f)[kQ], R (&g)[kQ]) {
    if (!(row_real<3>(c, r) && q.real)) {
      zero_row(f, g);
      return;
    }
    read_row<S, R>(buf(b), lane, f, g);
    first_collide<R, MODEL>(c, k, q, r, f, g);
  };
  // levels 2 and 3 of row r from the window below them, with the strip flux
  // of row 0 (counted once per level by the segment that owns row 0)
  auto next_level = [&](int r, const R (&cf)[kQ], const R (&cg)[kQ], const R (&nf)[kQ],
                        const R (&ng)[kQ], const R (&af)[3], const R (&ag)[3], R (&f)[kQ], R (&g)[kQ]) {
    second_collide<R, D, WALLS, MODEL>(c, k, q, r, cf, cg, nf, ng, af, ag, f, g);
    if (r == 0 && q.strip_flux) add_strip_flux<R>(c, k, q.x, g);
  };

  const int ys = D > 0 ? y0 : y1 - 1;
  const int ye = D > 0 ? y1 : y0 - 1;
  R c1f[kQ], c1g[kQ], n1f[kQ], n1g[kQ], a1f[3], a1g[3];  // level-1 window
  R c2f[kQ], c2g[kQ], n2f[kQ], n2g[kQ], a2f[3], a2g[3];  // level-2 window
  R c3f[kQ], c3g[kQ], n3f[kQ], n3g[kQ], a3f[3], a3g[3];  // level-3 window
  // prologue: level 1 of rows ys-3D .. ys+2D, level 2 of ys-2D .. ys+D,
  // level 3 of ys-D and ys; rows alternate between the two buffers
  issue(ys - 3 * D, 0);
  issue(ys - 2 * D, 1);
  wait_vm();
  level1(ys - 3 * D, 0, c1f, c1g);
  wait_lgkm();
  issue(ys - D, 0);
  level1(ys - 2 * D, 1, n1f, n1g);
  slide<D>(a1f, a1g, c1f, c1g, n1f, n1g);
  wait_vm();
  wait_lgkm();
  issue(ys, 1);
  level1(ys - D, 0, n1f, n1g);
  next_level(ys - 2 * D, c1f, c1g, n1f, n1g, a1f, a1g, c2f, c2g);
  slide<D>(a1f, a1g, c1f, c1g, n1f, n1g);
  wait_vm();
  wait_lgkm();
  issue(ys + D, 0);
  level1(ys, 1, n1f, n1g);
  next_level(ys - D, c1f, c1g, n1f, n1g, a1f, a1g, n2f, n2g);
  slide<D>(a2f, a2g, c2f, c2g, n2f, n2g);
  slide<D>(a1f, a1g, c1f, c1g, n1f, n1g);
  wait_vm();
  wait_lgkm();
  issue(ys + 2 * D, 1);
  level1(ys + D, 0, n1f, n1g);
  next_level(ys, c1f, c1g, n1f, n1g, a1f, a1g, n2f, n2g);
  next_level(ys - D, c2f, c2g, n2f, n2g, a2f, a2g, c3f, c3g);
  slide<D>(a2f, a2g, c2f, c2g, n2f, n2g);
  slide<D>(a1f, a1g, c1f, c1g, n1f, n1g);
  wait_vm();
  wait_lgkm();
  issue(ys + 3 * D, 0);
  level1(ys + 2 * D, 1, n1f, n1g);
  next_level(ys + D, c1f, c1g, n1f, n1g, a1f, a1g, n2f, n2g);
  next_level(ys, c2f, c2g, n2f, n2g, a2f, a2g, n3f, n3g);
  slide<D>(a3f, a3g, c3f, c3g, n3f, n3g);
  slide<D>(a2f, a2g, c2f, c2g, n2f, n2g);
  slide<D>(a1f, a1g, c1f, c1g, n1f, n1g);
  wait_vm();
  int b = 0;
  for (int y = ys; y != ye; y += D, b ^= 1) {
    // row y+3D is in buffer b; buffer b^1 (row y+2D) has been read
    wait_lgkm();
    if (y + D != ye) issue(y + 4 * D, b ^ 1);
    level1(y + 3 * D, b, n1f, n1g);
    next_level(y + 2 * D, c1f, c1g, n1f, n1g, a1f, a1g, n2f, n2g);
    next_level(y + D, c2f, c2g, n2f, n2g, a2f, a2g, n3f, n3g);
    R pf[kQ], pg[kQ];
    second_collide<R, D, WALLS, MODEL>(c, k, q, y, c3f, c3g, n3f, n3g, a3f, a3g, pf, pg);
    wait_vm();
    emit<S, R, WALLS>(c, k, B, q, y, pf, pg);
    slide<D>(a3f, a3g, c3f, c3g, n3f, n3g);
    slide<D>(a2f, a2g, c2f, c2g, n2f, n2g);
    slide<D>(a1f, a1g, c1f, c1g, n1f, n1g);
  }
}

template <typename S, typename R, int MODEL>
__global__ __launch_bounds__(kWave)
__attribute__((amdgpu_waves_per_eu(2))) void k_step4(CavDev c, int strips_x, int nseg, int seg_rows,
                                                     int order) {
  __shared__ S lds[2 * kPlanes * kWave];
  const int lane = threadIdx.x & (kWave - 1);
  const int w = tile_of(blockIdx.x, gridDim.x, order & 1, (order & 2) && (c.parity & 1));
  if (w >= strips_x * nseg) return;  // uniform per wavefront; no barriers follow
  const int strip = w % strips_x, seg = w / strips_x;
  const int x0 = strip * kStrip4Cols;
  const int y0 = seg * seg_rows;
  const int y1 = min(y0 + seg_rows, c.ny);
  const Col q = make_col<3>(c, x0 - 3 + lane, lane, y0);
  const Coef<R> k(c);
  const S *__restrict__ A = static_cast<const S *>(c.parity ? c.pop[1] : c.pop[0]);
  S *__restrict__ B = static_cast<S *>(c.parity ? c.pop[0] : c.pop[1]);
  const bool down = (order & 4) && (seg & 1);
  const bool inner = interior_segment<3>(c, x0, y0, y1);
  if (down) {
    if (inner)
      walk4_staged<S, R, -1, false, MODEL>(c, k, A, B, q, y0, y1, x0, lds);
    else
      walk4_staged<S, R, -1, true, MODEL>(c, k, A, B, q, y0, y1, x0, lds);
  } else {
    if (inner)
      walk4_staged<S, R, +1, false, MODEL>(c, k, A, B, q, y0, y1, x0, lds);
    else
      walk4_staged<S, R, +1, true, MODEL>(c, k, A, B, q, y0, y1, x0, lds);
  }
}

hipError_t dispatch4(const CavDev &c, const LaunchCfg &cfg, hipStream_t s) {
  if (cfg.seg4 < 1 || cfg.seg4 > kMaxSegmentRows) return hipErrorInvalidValue;
  const int strips_x = (c.nx + kStrip4Cols - 1) / kStrip4Cols;
  const int nseg = (c.ny + cfg.seg4 - 1) / cfg.seg4;
  const int order = (cfg.xcd ? 1 : 0) | (cfg.reverse ? 2 : 0) | (cfg.zigzag ? 4 : 0);
  with_kernel_model(c.kmodel, [&](auto m) {
    hipLaunchKernelGGL((k_step4<float, float, decltype(m)::value>), dim3(strips_x * nseg), dim3(kWave), 0, s,
                       c, strips_x, nseg, cfg.seg4, order);
    return 0;
  });
  return hipGetLastError();
}

// The same three-step walk with the level-2 window kept in LDS instead of
// registers, for FP64, whose two register windows exceed the register file.
// Rows are loaded directly (the LDS holds the window, not staged rows).  The
// window is a ring of two level-2 rows per wavefront, row r in slot r & 1:
// iteration y reads the populations of row y-D that move along the walk from
// slot y-D, then overwrites that slot with row y+D; row y is read from its
// slot when the third step gathers.  Each lane reads and writes only its own
// column of a slot, and LDS operations of a wavefront complete in order, so
// no barrier is needed.
template <typename S, typename R, int D, bool WALLS, int MODEL, int STEPS = 3, bool PIPE = true>
__device__ __forceinline__ void walk3_ring(const CavDev &c, const Rates<R> &k, const S *__restrict__ A,
                                           S *__restrict__ B, const Col &q, int y0, int y1, R *ring) {
  const int lane = threadIdx.x & (kWave - 1);
  auto slot = [&](int r) { return ring + (r & 1) * (kPlanes * kWave) + lane; };
  auto put = [&](int r, const R (&f)[kQ], const R (&g)[kQ]) {
    R *p = slot(r);
#pragma unroll
    for (int i = 0; i < kQ; ++i) {
      p[i * kWave] = f[i];
      p[(kQ + i) * kWave] = g[i];
    }
  };
  auto get = [&](int r, R (&f)[kQ], R (&g)[kQ]) {
    const R *p = slot(r);
#pragma unroll
    for (int i = 0; i < kQ; ++i) {
      f[i] = p[i * kWave];
      g[i] = p[(kQ + i) * kWave];
    }
  };
  auto get_along = [&](int r, R (&af)[3], R (&ag)[3]) {
    constexpr int a0 = D > 0 ? 2 : 4, a1 = D > 0 ? 5 : 7, a2 = D > 0 ? 6 : 8;
    const R *p = slot(r);
    af[0] = p[a0 * kWave]; af[1] = p[a1 * kWave]; af[2] = p[a2 * kWave];
    ag[0] = p[(kQ + a0) * kWave]; ag[1] = p[(kQ + a1) * kWave]; ag[2] = p[(kQ + a2) * kWave];
  };
  // level 1 in two halves: the loads of a row, and its collision once they are
  // in.  The loads sit outside every branch, so the wavefront need not wait
  // for them where they are issued: a lane whose column does not exist loads
  // column 0 of the row, and a row that does not exist loads the nearest row
  // of the cavity; such values are never used (the links that would read them
  // are reflected at the wall), and rows that do not exist are zeroed.
  const int lcol = q.real ? q.xw : 0;
  auto load1 = [&](int r, R (&f)[kQ], R (&g)[kQ]) {
    const int rr = row_real<2>(c, r) ? row_wrap<2>(c, r) : min(max(r, 0), c.ny - 1);
    load_natural<S, R>(A, c.plane, cell_base(c, lcol, rr), f, g);
  };
  auto collide1 = [&](int r, R (&f)[kQ], R (&g)[kQ]) {
    if (row_real<2>(c, r))  // wavefront-uniform
      first_collide<R, MODEL>(c, k, q, r, f, g);
    else
      zero_row(f, g);
  };
  auto level1 = [&](int r, R (&f)[kQ], R (&g)[kQ]) {
    load1(r, f, g);
    collide1(r, f, g);
  };
  auto level2 = [&](int r, const R (&cf)[kQ], const R (&cg)[kQ], const R (&nf)[kQ],
                    const R (&ng)[kQ], const R (&af)[3], const R (&ag)[3], R (&f)[kQ], R (&g)[kQ]) {
    second_collide<R, D, WALLS, MODEL>(c, k, q, r, cf, cg, nf, ng, af, ag, f, g);
    if (r == 0 && q.strip_flux) add_strip_flux<R>(c, k, q.x, g);
  };

  const int ys = D > 0 ? y0 : y1 - 1;
  const int ye = D > 0 ? y1 : y0 - 1;
  R c1f[kQ], c1g[kQ], n1f[kQ], n1g[kQ], a1f[3], a1g[3];  // level-1 window
  {
    R t2f[kQ], t2g[kQ];
    level1(ys - 2 * D, c1f, c1g);
    level1(ys - D, n1f, n1g);
    slide<D>(a1f, a1g, c1f, c1g, n1f, n1g);
    level1(ys, n1f, n1g);
    level2(ys - D, c1f, c1g, n1f, n1g, a1f, a1g, t2f, t2g);
    put(ys - D, t2f, t2g);
    slide<D>(a1f, a1g, c1f, c1g, n1f, n1g);
    level1(ys + D, n1f, n1g);
    level2(ys, c1f, c1g, n1f, n1g, a1f, a1g, t2f, t2g);
    put(ys, t2f, t2g);
    slide<D>(a1f, a1g, c1f, c1g, n1f, n1g);
  }
  // PIPE: the loads of each walk row are issued one iteration early, before
  // the third step and the stores of the previous row, so they overlap that
  // work instead of being waited for right after their issue; the last
  // iteration, which has no next row, is peeled off so that the loop always
  // loads.  This holds one row more in registers (the batched kernel, whose
  // item loop needs more of them, loads each row when it collides it).
  auto iteration = [&](int y, auto load_next) {
    R n2f[kQ], n2g[kQ];
    if constexpr (!PIPE) load1(y + 2 * D, n1f, n1g);
    collide1(y + 2 * D, n1f, n1g);
    level2(y + D, c1f, c1g, n1f, n1g, a1f, a1g, n2f, n2g);
    slide<D>(a1f, a1g, c1f, c1g, n1f, n1g);
    if constexpr (STEPS == 3) {
      R a2f[3], a2g[3];
      get_along(y - D, a2f, a2g);
      put(y + D, n2f, n2g);  // the slot of row y-D
      R pf[kQ], pg[kQ];
      if constexpr (PIPE && decltype(load_next)::value) load1(y + 3 * D, n1f, n1g);
      third_collide<R, D, WALLS, MODEL>(c, k, q, y, slot(y), n2f, n2g, a2f, a2g, pf, pg);
      emit<S, R, WALLS>(c, k, B, q, y, pf, pg);
    } else {
      R c2f[kQ], c2g[kQ];
      get(y, c2f, c2g);
      put(y + D, n2f, n2g);
      if constexpr (PIPE && decltype(load_next)::value) load1(y + 3 * D, n1f, n1g);
      emit<S, R, WALLS, false>(c, k, B, q, y, c2f, c2g);
    }
  };
  if constexpr (PIPE) load1(ys + 2 * D, n1f, n1g);
  for (int y = ys; y != ye - D; y += D) iteration(y, std::true_type{});
  iteration(ye - D, std::false_type{});
}

// The three-step walk for either precision, direction and wall case.
template <typename S, typename R, int MODEL, int STEPS, bool PIPE = false>
__device__ __forceinline__ void walk3(bool down, bool inner, const CavDev &c, const Rates<R> &k,
                                      const S *__restrict__ A, S *__restrict__ B, const Col &q, int y0,
                                      int y1, int x0, R *mine) {
  if constexpr (sizeof(R) == 8) {
    // FP64: level-2 ring of two rows of R
    if (down) {
      if (inner)
        walk3_ring<S, R, -1, false, MODEL, STEPS, PIPE>(c, k, A, B, q, y0, y1, mine);
      else
        walk3_ring<S, R, -1, true, MODEL, STEPS, PIPE>(c, k, A, B, q, y0, y1, mine);
    } else {
      if (inner)
        walk3_ring<S, R, +1, false, MODEL, STEPS, PIPE>(c, k, A, B, q, y0, y1, mine);
      else
        walk3_ring<S, R, +1, true, MODEL, STEPS, PIPE>(c, k, A, B, q, y0, y1, mine);
    }
  } else {
    // FP32: two staged rows of S
    S *bufs = reinterpret_cast<S *>(mine);
    if (down) {
      if (inner)
        walk3_staged<S, R, -1, false, MODEL, STEPS>(c, k, A, B, q, y0, y1, x0, bufs);
      else
        walk3_staged<S, R, -1, true, MODEL, STEPS>(c, k, A, B, q, y0, y1, x0, bufs);
    } else {
      if (inner)
        walk3_staged<S, R, +1, false, MODEL, STEPS>(c, k, A, B, q, y0, y1, x0, bufs);
      else
        walk3_staged<S, R, +1, true, MODEL, STEPS>(c, k, A, B, q, y0, y1, x0, bufs);
    }
  }
}

template <typename S, typename R, int MODEL>
__global__ __launch_bounds__(kStep3Waves * kWave)
__attribute__((amdgpu_waves_per_eu(2))) void k_step3(CavDev c, int strips_x, int nseg, int seg_rows,
                                                     int order) {
  __shared__ R lds[kStep3Waves * 2 * kPlanes * kWave];
  const int lane = threadIdx.x & (kWave - 1);
  const int wid = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
  const int b = tile_of(blockIdx.x, gridDim.x, order & 1, (order & 2) && (c.parity & 1));
  const int w = b * kStep3Waves + wid;
  if (w >= strips_x * nseg) return;  // uniform per wavefront; no barriers follow
  const int strip = w % strips_x, seg = w / strips_x;
  const int x0 = strip * kStrip3Cols;
  const int y0 = seg * seg_rows;
  const int y1 = min(y0 + seg_rows, c.ny);
  const Col q = make_col<2>(c, x0 - 2 + lane, lane, y0);
  const Coef<R> k(c);
  const S *__restrict__ A = static_cast<const S *>(c.parity ? c.pop[1] : c.pop[0]);
  S *__restrict__ B = static_cast<S *>(c.parity ? c.pop[0] : c.pop[1]);
  const bool down = (order & 4) && (seg & 1);
  R *mine = lds + wid * 2 * kPlanes * kWave;
  walk3<S, R, MODEL, 3, true>(down, interior_segment<2>(c, x0, y0, y1), c, k, A, B, q, y0, y1, x0, mine);
}

template <typename S, typename R>
hipError_t dispatch3(const CavDev &c, const LaunchCfg &cfg, hipStream_t s) {
  if (cfg.seg3 < 1 || cfg.seg3 > kMaxSegmentRows) return hipErrorInvalidValue;
  const int strips_x = (c.nx + kStrip3Cols - 1) / kStrip3Cols;
  const int nseg = (c.ny + cfg.seg3 - 1) / cfg.seg3;
  const int waves = strips_x * nseg;
  const dim3 grid((waves + kStep3Waves - 1) / kStep3Waves);
  const int order = (cfg.xcd ? 1 : 0) | (cfg.reverse ? 2 : 0) | (cfg.zigzag ? 4 : 0);
  with_kernel_model(c.kmodel, [&](auto m) {
    hipLaunchKernelGGL((k_step3<S, R, decltype(m)::value>), grid, dim3(kStep3Waves * kWave), 0, s, c,
                       strips_x, nseg, cfg.seg3, order);
    return 0;
  });
  return hipGetLastError();
}

// Batched two-step launch: each wavefront takes items (one strip segment of
// one cavity) from its XCD's contiguous band of the item list, so the
// segments of a cavity share that XCD's L2.  Cavity state comes from the
// device array, so a captured launch stays valid when cavities join or
// leave.  The storage parity in launch j is the chunk-start parity flipped j
// times: every earlier launch of the chunk advanced the cavity.
template <typename S, typename R, bool STAGED, int MODEL>
__global__ __launch_bounds__(STAGED ? kStagedWaves * kWave : kDirectWaves * kWave)
__attribute__((amdgpu_waves_per_eu(2))) void k_step2_batch(const CavDev *__restrict__ cavs,
                                                           const BatchTile *__restrict__ items,
                                                           const int32_t *__restrict__ hdr,
                                                           int item_cap, int seg_rows,
                                                           int launch_index, int order,
                                                           int32_t *__restrict__ err) {
  constexpr int waves = STAGED ? kStagedWaves : kDirectWaves;
  __shared__ S lds[STAGED ? waves * 2 * kPlanes * kWave : 1];
  const int first = hdr[0], n = hdr[1];
  if (!batch_header_ok(first, n, item_cap)) {
    if (threadIdx.x == 0) *err = kErrBatchHeader;
    return;
  }
  const int lane = threadIdx.x & (kWave - 1);
  const int wid = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
  const int xcd = blockIdx.x % kXcds, lb = blockIdx.x / kXcds;
  const int nbx = (gridDim.x - xcd + kXcds - 1) / kXcds;
  const int t0 = (int)((int64_t)n * xcd / kXcds);
  const int t1 = (int)((int64_t)n * (xcd + 1) / kXcds);
  for (int t = t0 + lb * waves + wid; t < t1; t += nbx * waves) {  // uniform per wavefront
    const BatchTile it = items[first + t];
    CavDev c = cavs[it.cav];
    const int a = c.active_steps;
    if (2 * launch_index + 1 > a) continue;
    c.parity ^= (launch_index & 1);
    const int y0 = it.y0;
    const int y1 = min(y0 + seg_rows, c.ny);
    const Coef<R, true> k(c);
    const S *__restrict__ A = static_cast<const S *>(c.parity ? c.pop[1] : c.pop[0]);
    S *__restrict__ B = static_cast<S *>(c.parity ? c.pop[0] : c.pop[1]);
    if (2 * launch_index + 2 <= a) {
      const Col q = make_col(c, it.x0 - 1 + lane, lane, y0);
      const bool down = (order & 4) && (it.pad & 1);
      if constexpr (STAGED) {
        S *bufs = lds + wid * 2 * kPlanes * kWave;
        const bool inner = interior_segment(c, it.x0, y0, y1);
        if (down) {
          if (inner)
            walk_staged<S, R, -1, false, MODEL>(c, k, A, B, q, y0, y1, it.x0, bufs);
          else
            walk_staged<S, R, -1, true, MODEL>(c, k, A, B, q, y0, y1, it.x0, bufs);
        } else {
          if (inner)
            walk_staged<S, R, +1, false, MODEL>(c, k, A, B, q, y0, y1, it.x0, bufs);
          else
            walk_staged<S, R, +1, true, MODEL>(c, k, A, B, q, y0, y1, it.x0, bufs);
        }
      } else {
        if (down)
          walk_direct<S, R, -1, MODEL>(c, k, A, B, q, y0, y1);
        else
          walk_direct<S, R, +1, MODEL>(c, k, A, B, q, y0, y1);
      }
    } else {
      // the odd last step of the chunk: single two-lattice steps of the
      // segment's owned cells
      const int x = it.x0 - 1 + lane;
      if (lane >= 1 && lane <= kStripCols && x < c.nx)
        for (int y = y0; y < y1; ++y) update_cell<S, R, MODEL>(c, k, 2, x, y);
    }
  }
}

// Batched three-step launch: items are 60-column strip segments of the
// three-step cavities, taken as in the two-step batched launch.  Launch j of
// a chunk advances a cavity by three steps while 3j + 3 <= active_steps, and
// by the one or two steps left of the chunk otherwise (a walk that stores
// level 2, or single steps of the segment's owned cells).
template <typename S, typename R, int MODEL>
__global__ __launch_bounds__(kStagedWaves * kWave)
__attribute__((amdgpu_waves_per_eu(2))) void k_step3_batch(const CavDev *__restrict__ cavs,
                                                           const BatchTile *__restrict__ items,
                                                           const int32_t *__restrict__ hdr,
                                                           int item_cap, int seg_rows,
                                                           int launch_index, int order,
                                                           int32_t *__restrict__ err) {
  __shared__ R lds[kStagedWaves * 2 * kPlanes * kWave];
  const int first = hdr[0], n = hdr[1];
  if (!batch_header_ok(first, n, item_cap)) {
    if (threadIdx.x == 0) *err = kErrBatchHeader;
    return;
  }
  const int lane = threadIdx.x & (kWave - 1);
  const int wid = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
  const int xcd = blockIdx.x % kXcds, lb = blockIdx.x / kXcds;
  const int nbx = (gridDim.x - xcd + kXcds - 1) / kXcds;
  const int t0 = (int)((int64_t)n * xcd / kXcds);
  const int t1 = (int)((int64_t)n * (xcd + 1) / kXcds);
  R *mine = lds + wid * 2 * kPlanes * kWave;
  for (int t = t0 + lb * kStagedWaves + wid; t < t1; t += nbx * kStagedWaves) {  // uniform per wavefront
    const BatchTile it = items[first + t];
    CavDev c = cavs[it.cav];
    const int left = c.active_steps - 3 * launch_index;
    if (left <= 0) continue;
    c.parity ^= (launch_index & 1);
    const int y0 = it.y0;
    const int y1 = min(y0 + seg_rows, c.ny);
    const Coef<R, true> k(c);
    const S *__restrict__ A = static_cast<const S *>(c.parity ? c.pop[1] : c.pop[0]);
    S *__restrict__ B = static_cast<S *>(c.parity ? c.pop[0] : c.pop[1]);
    const Col q = make_col<2>(c, it.x0 - 2 + lane, lane, y0);
    if (left == 1) {
      if (q.owner)
        for (int y = y0; y < y1; ++y) update_cell<S, R, MODEL>(c, k, 2, q.x, y);
      continue;
    }
    const bool down = (order & 4) && (it.pad & 1);
    const bool inner = interior_segment<2>(c, it.x0, y0, y1);
    if (left >= 3)
      walk3<S, R, MODEL, 3>(down, inner, c, k, A, B, q, y0, y1, it.x0, mine);
    else
      walk3<S, R, MODEL, 2>(down, inner, c, k, A, B, q, y0, y1, it.x0, mine);
  }
}

template <typename S, typename R>
hipError_t dispatch3_batch(const CavDev *cavs, const BatchTile *items, const int32_t *hdr, int item_cap,
                           int model, const LaunchCfg &cfg, int launch_index, int grid, int32_t *err,
                           hipStream_t s) {
  if (cfg.seg3 < 1 || cfg.seg3 > kMaxSegmentRows) return hipErrorInvalidValue;
  const int order = cfg.zigzag ? 4 : 0;
  with_kernel_model(model, [&](auto m) {
    hipLaunchKernelGGL((k_step3_batch<S, R, decltype(m)::value>), dim3(grid), dim3(kStagedWaves * kWave), 0,
                       s, cavs, items, hdr, item_cap, cfg.seg3, launch_index, order, err);
    return 0;
  });
  return hipGetLastError();
}

template <typename S, typename R, bool STAGED>
hipError_t dispatch_batch(const CavDev *cavs, const BatchTile *items, const int32_t *hdr,
                          int item_cap, int model, const LaunchCfg &cfg, int launch_index,
                          int grid, int32_t *err, hipStream_t s) {
  if (cfg.seg < 1 || cfg.seg > kMaxSegmentRows) return hipErrorInvalidValue;
  const int per_block = STAGED ? kStagedWaves : kDirectWaves;
  const int order = cfg.zigzag ? 4 : 0;
  with_kernel_model(model, [&](auto m) {
    hipLaunchKernelGGL((k_step2_batch<S, R, STAGED, decltype(m)::value>), dim3(grid),
                       dim3(per_block * kWave), 0, s, cavs, items, hdr, item_cap, cfg.seg,
                       launch_index, order, err);
    return 0;
  });
  return hipGetLastError();
}

}  // namespace

int step2_batch_grid(int num_cus) {
  // four 2-wavefront workgroups (or two 4-wavefront ones) per CU
  return num_cus * 4;
}

hipError_t launch_step2_batch(const CavDev *cavs_dev, const BatchTile *items_dev,
                              const int32_t *hdr_dev, int item_cap, int precision, int model,
                              const LaunchCfg &cfg, int launch_index, int grid, int32_t *err_dev,
                              hipStream_t s) {
  if (cfg.staged)
    return precision == 0
               ? dispatch_batch<double, double, true>(cavs_dev, items_dev, hdr_dev, item_cap, model,
                                                      cfg, launch_index, grid, err_dev, s)
               : dispatch_batch<float, float, true>(cavs_dev, items_dev, hdr_dev, item_cap, model,
                                                    cfg, launch_index, grid, err_dev, s);
  return precision == 0
             ? dispatch_batch<double, double, false>(cavs_dev, items_dev, hdr_dev, item_cap, model,
                                                     cfg, launch_index, grid, err_dev, s)
             : dispatch_batch<float, float, false>(cavs_dev, items_dev, hdr_dev, item_cap, model,
                                                   cfg, launch_index, grid, err_dev, s);
}

hipError_t launch_step3_batch(const CavDev *cavs_dev, const BatchTile *items_dev,
                              const int32_t *hdr_dev, int item_cap, int precision, int model,
                              const LaunchCfg &cfg, int launch_index, int grid, int32_t *err_dev,
                              hipStream_t s) {
  return precision == 0 ? dispatch3_batch<double, double>(cavs_dev, items_dev, hdr_dev, item_cap, model,
                                                          cfg, launch_index, grid, err_dev, s)
                        : dispatch3_batch<float, float>(cavs_dev, items_dev, hdr_dev, item_cap, model,
                                                        cfg, launch_index, grid, err_dev, s);
}

namespace {

template <typename K>
int resident_waves(K kernel, int block_waves) {
  int blocks = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&blocks, reinterpret_cast<const void *>(kernel),
                                                   block_waves * kWave, 0) != hipSuccess) {
    (void)hipGetLastError();
    return 0;
  }
  return blocks * block_waves;
}

template <typename S, typename R>
int fused_waves(int steps, int kmodel, bool staged) {
  return with_kernel_model(kmodel, [&](auto m) {
    constexpr int M = decltype(m)::value;
    if (steps == 2)
      return staged ? resident_waves(&k_step2<S, R, true, M>, kStagedWaves)
                    : resident_waves(&k_step2<S, R, false, M>, kDirectWaves);
    if (steps == 3) return resident_waves(&k_step3<S, R, M>, kStep3Waves);
    if constexpr (sizeof(R) == 4) {
      if (steps == 4) return resident_waves(&k_step4<S, R, M>, 1);
    }
    return 0;
  });
}

}  // namespace

int fused_waves_per_cu(int precision, int steps, int kmodel, bool staged) {
  return precision == 0 ? fused_waves<double, double>(steps, kmodel, staged)
                        : fused_waves<float, float>(steps, kmodel, staged);
}

hipError_t launch_step4(const CavDev &c, int precision, const LaunchCfg &cfg, hipStream_t s) {
  return precision == 0 ? hipErrorInvalidValue : dispatch4(c, cfg, s);
}

hipError_t launch_step3(const CavDev &c, int precision, const LaunchCfg &cfg, hipStream_t s) {
  return precision == 0 ? dispatch3<double, double>(c, cfg, s) : dispatch3<float, float>(c, cfg, s);
}

hipError_t launch_step2(const CavDev &c, int precision, const LaunchCfg &cfg, hipStream_t s) {
  if (cfg.staged)
    return precision == 0 ? dispatch<double, double, true>(c, cfg, s)
                          : dispatch<float, float, true>(c, cfg, s);
  return precision == 0 ? dispatch<double, double, false>(c, cfg, s)
                        : dispatch<float, float, false>(c, cfg, s);
}

}  // namespace lbm
