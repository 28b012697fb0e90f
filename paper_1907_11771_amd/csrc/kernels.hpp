// Step kernels of the extrapolated GBS macro step (streaming form).
//
// One launch of lf_kernel advances every active sequence j (N_j >= s) by one
// leap-frog step, y_{s+1} = y_{s-1} + 2 h_j f(t_0 + s h_j, y_s) (Sect. 2.1,
// eq. GBS), over the whole grid: blockIdx.y selects the sequence,
// blockIdx.z the right-hand side.  At s = N_j the level y_{N+1} is not
// stored; instead the averaging y* = (y_{N-1} + 2 y_N + y_{N+1}) / 4 and the
// weighted combination (Sect. 3.2) are applied in FP64 into the accumulator.
// Sequences finish in ascending N, so the combination is summed in that
// order.  first_kernel evaluates f(t_0, y_0) once and writes
// y_1 = y_0 + h_j f(t_0, y_0) for every sequence (Sect. 3.6).
#pragma once

#include "stencil.hpp"

namespace gbs {

constexpr int OP_ADV1D = GBS_ADVECT1D;
constexpr int OP_AC2D = GBS_ACOUSTIC2D;
constexpr int OP_AC3D = GBS_ACOUSTIC3D;

template <int OP>
struct NFields;
template <> struct NFields<OP_ADV1D> { static constexpr int F = 1; };
template <> struct NFields<OP_AC2D> { static constexpr int F = 3; };
template <> struct NFields<OP_AC3D> { static constexpr int F = 4; };

// f(t, y) at grid point (x, y, z) of one right-hand side (without sources).
// Fields (p, v_x, v_y[, v_z]):  f_p = -c^2 div v,  f_v = -grad p;
// advection: f_u = -u_x.
template <typename T, int ORDER, int OP>
__device__ __forceinline__ void eval_rhs(const T* __restrict__ s, int x, int y, int z,
                                         const Geometry& g, T c2, T invx, T invy, T invz,
                                         T* f) {
  if constexpr (OP == OP_ADV1D) {
    f[0] = -(invx * dsum<T, ORDER>(s, x, g.nx, 1));
  } else if constexpr (OP == OP_AC2D) {
    const int64_t row = (int64_t)y * g.nx;
    const T* p = s;
    const T* vx = s + g.field;
    const T* vy = s + 2 * g.field;
    const T dvx = invx * dsum<T, ORDER>(vx + row, x, g.nx, 1);
    const T dvy = invy * dsum<T, ORDER>(vy + x, y, g.ny, g.nx);
    f[0] = -(c2 * (dvx + dvy));
    f[1] = -(invx * dsum<T, ORDER>(p + row, x, g.nx, 1));
    f[2] = -(invy * dsum<T, ORDER>(p + x, y, g.ny, g.nx));
  } else {
    const int64_t plane = (int64_t)g.nx * g.ny;
    const int64_t row = (int64_t)z * plane + (int64_t)y * g.nx;
    const int64_t col = (int64_t)z * plane + x;
    const int64_t pil = (int64_t)y * g.nx + x;
    const T* p = s;
    const T* vx = s + g.field;
    const T* vy = s + 2 * g.field;
    const T* vz = s + 3 * g.field;
    const T dvx = invx * dsum<T, ORDER>(vx + row, x, g.nx, 1);
    const T dvy = invy * dsum<T, ORDER>(vy + col, y, g.ny, g.nx);
    const T dvz = invz * dsum<T, ORDER>(vz + pil, z, g.nz, plane);
    f[0] = -(c2 * ((dvx + dvy) + dvz));
    f[1] = -(invx * dsum<T, ORDER>(p + row, x, g.nx, 1));
    f[2] = -(invy * dsum<T, ORDER>(p + col, y, g.ny, g.nx));
    f[3] = -(invz * dsum<T, ORDER>(p + pil, z, g.nz, plane));
  }
}

__device__ __forceinline__ void decompose(int64_t idx, const Geometry& g, int& x, int& y, int& z) {
  x = (int)(idx % g.nx);
  const int64_t r = idx / g.nx;
  y = (int)(r % g.ny);
  z = (int)(r / g.ny);
}

template <typename T>
__device__ __forceinline__ T source_term(const SrcDesc* src, int nsrc, int64_t rhs, int64_t idx,
                                         double amp) {
  T add = T(0);
  for (int k = 0; k < nsrc; ++k)
    if (src[k].rhs == rhs && src[k].idx == idx) add += (T)(src[k].w * amp);
  return add;
}

template <typename T, int ORDER, int OP>
__global__ __launch_bounds__(256) void lf_kernel(const StepArgs<T> a) {
  constexpr int F = NFields<OP>::F;
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= a.g.field) return;
  const SeqDesc<T>& d = a.seq[blockIdx.y];
  const int64_t rhs = blockIdx.z;
  const int64_t base = rhs * a.g.state;
  int x, y, z;
  decompose(idx, a.g, x, y, z);
  const T c2 = a.c2f ? a.c2f[idx] : a.c2c;
  T f[F];
  eval_rhs<T, ORDER, OP>(d.cur + base, x, y, z, a.g, c2, a.invx, a.invy, a.invz, f);
  if (a.g.nsrc) f[0] += source_term<T>(a.src, a.g.nsrc, rhs, idx, d.amp);
#pragma unroll
  for (int q = 0; q < F; ++q) {
    const int64_t e = base + q * a.g.field + idx;
    const T o = d.old[e];
    const T nw = o + d.h2 * f[q];
    if (!(d.mode & MODE_LAST)) {
      d.out[e] = nw;
    } else {
      const double ys = 0.25 * (((double)o + 2.0 * (double)d.cur[e]) + (double)nw);
      double v = d.cw * ys;
      if (!(d.mode & MODE_FIRST)) v = a.acc[e] + v;
      if (d.mode & MODE_FINAL) a.yout[e] = (T)v;
      else a.acc[e] = v;
    }
  }
}

template <typename T, int ORDER, int OP>
__global__ __launch_bounds__(256) void first_kernel(const FirstArgs<T> a) {
  constexpr int F = NFields<OP>::F;
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= a.g.field) return;
  const int64_t rhs = blockIdx.z;
  const int64_t base = rhs * a.g.state;
  int x, y, z;
  decompose(idx, a.g, x, y, z);
  const T c2 = a.c2f ? a.c2f[idx] : a.c2c;
  T f[F];
  eval_rhs<T, ORDER, OP>(a.y0 + base, x, y, z, a.g, c2, a.invx, a.invy, a.invz, f);
  if (a.g.nsrc) f[0] += source_term<T>(a.src, a.g.nsrc, rhs, idx, a.amp);
#pragma unroll
  for (int q = 0; q < F; ++q) {
    const int64_t e = base + q * a.g.field + idx;
    const T v0 = a.y0[e];
    for (int j = 0; j < a.nseq; ++j) a.out[j][e] = v0 + a.h[j] * f[q];
  }
}

}  // namespace gbs
