// Auxiliary kernels of the B-TriRT melting library: initial states, raw
// state load/save, macroscopic fields and the FP64 compensated reductions
// behind the diagnostics (melt fraction, total enthalpy, strip flux, mass).
#include "lbm_device.h"

namespace lbm {
namespace {

using namespace dev;

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
  const int64_t idx = cell_base(c, x, y);
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
  const int64_t idx = cell_base(c, x, y);
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
  const int64_t idx = cell_base(c, x, y);
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
  // fluid velocity of the solid model: scaled by fl, held by the drag
  // (u = (fl^3 + eps)/D (j + F/2)/rho0, D = fl^3 + eps + C (1 - fl)^2 / 2),
  // or free (bounce-back model)
  double s = fl;
  if (c.solid_model == kSolidDarcy) {
    const double fl3e = fl * fl * fl + c.darcy_eps;
    s = fl3e / (fl3e + 0.5 * c.darcy_c * (1.0 - fl) * (1.0 - fl));
  } else if (c.solid_model == kSolidPbb) {
    s = 1.0;
  }
  m.ux = s * jx * c.inv_rho0;
  m.uy = s * (jy + 0.5 * Fy) * c.inv_rho0;
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

}  // namespace

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

// Streaming ceiling of the blocked lattice layout: each wavefront reads one
// 64-cell chunk of 18 FP64 planes (9 KiB) and writes it to the other buffer
// (the two-lattice pattern) or back into the same chunk (in place), with the
// step kernels' order: workgroups of four wavefronts in contiguous bands per
// XCD, walked backwards on odd launches.  No lattice arithmetic: it measures
// what the memory system gives that access pattern.
__global__ __launch_bounds__(256) void k_stream(const double *__restrict__ src, double *__restrict__ dst,
                                                int64_t chunks, int back) {
  const int wid = threadIdx.x >> 6, lane = threadIdx.x & (kWave - 1);
  const int64_t t = (int64_t)tile_of(blockIdx.x, gridDim.x, true, back != 0) * 4 + wid;
  if (t >= chunks) return;
  const double *a = src + t * (kPlanes * kWave) + lane;
  double *b = dst + t * (kPlanes * kWave) + lane;
  double v[kPlanes];
#pragma unroll
  for (int i = 0; i < kPlanes; ++i) v[i] = a[i * kWave];
#pragma unroll
  for (int i = 0; i < kPlanes; ++i) b[i * kWave] = v[i] + 1.0;
}

hipError_t launch_stream(const double *src, double *dst, int64_t chunks, int back, hipStream_t s) {
  const int64_t blocks = (chunks + 3) / 4;
  if (chunks < 1 || blocks > INT32_MAX) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_stream, dim3((unsigned)blocks), dim3(256), 0, s, src, dst, chunks, back);
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
