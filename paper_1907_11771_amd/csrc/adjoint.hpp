// Discrete adjoint of one extrapolated GBS macro step for the acoustic
// operators (2-D and 3-D), and the receiver gather / injection kernels.
//
// The paper defines the forward step only (Sect. 2.1, eq. GBS; Sect. 3.2).
// For f(t, y) = A y + s(t) (A linear in y and, through C = diag(c^2), in the
// coefficient field) the transpose of one sequence is its recurrence run
// backwards.  With lambda_n the adjoint of level y_n and w = c_j ybar_out:
//   lambda_{N+1} = w/4, lambda_N = w/2, lambda_{N-1} = w/4 (averaging),
//   for n = N..1:  lambda_n += 2h A^T lambda_{n+1};  lambda_{n-1} += lambda_{n+1},
//   ybar_0 += lambda_0 + lambda_1,  Fbar_0 += h lambda_1   (forward Euler),
// and once for all sequences ybar_0 += A^T Fbar_0 (shared first evaluation).
// Two buffers carry (lambda_{n+1} final, lambda_n partial): one step reads
// the first at the stencil's neighbours and updates the second in place,
// then the roles swap, as in the forward leap-frog.  The gradient with
// respect to c^2 collects a * lambda_p * (-div v_n) for every application of
// A with factor a (2h, or h_j for the shared first evaluation), in FP64.
//
// Periodic centred differences are antisymmetric (D^T = -D), so
//   (A^T w)_p = sum_k D_k w_{v_k},   (A^T w)_{v_k} = D_k (c^2 w_p).
#pragma once

#include "kernels.hpp"

namespace gbs {

// sum_m W_m (c2[i+m] u[i+m] - c2[i-m] u[i-m]) along one axis (product
// formed at each neighbour).
template <typename T, int ORDER>
__device__ __forceinline__ T dsum_c2(const T* __restrict__ u, const T* __restrict__ c2f, T c2c,
                                     int i, int n, int64_t stride) {
  T s = T(0);
#pragma unroll
  for (int k = 0; k < Fd<ORDER>::R; ++k) {
    const int64_t iu = (int64_t)wrap(i + k + 1, n) * stride;
    const int64_t id = (int64_t)wrap(i - k - 1, n) * stride;
    const T up = (c2f ? c2f[iu] : c2c) * u[iu];
    const T dn = (c2f ? c2f[id] : c2c) * u[id];
    s += Fd<ORDER>::template w<T>(k) * (up - dn);
  }
  return s;
}

// A^T w at (x, y, z) of one right-hand side w (fields p, v...), and -div v
// of a state s at the same point.
template <typename T, int ORDER, int OP>
__device__ __forceinline__ void eval_AT(const T* __restrict__ w, const T* __restrict__ c2f, T c2c,
                                        int x, int y, int z, const Geometry& g, T invx, T invy,
                                        T invz, T* out) {
  constexpr int D = OP == OP_AC2D ? 2 : 3;
  const int64_t plane = (int64_t)g.nx * g.ny;
  const int64_t xline = (int64_t)z * plane + (int64_t)y * g.nx;
  const int64_t yline = (int64_t)z * plane + x;
  const int64_t zline = (int64_t)y * g.nx + x;
  const T* p = w;
  const T* c2x = c2f ? c2f + xline : nullptr;
  const T* c2y = c2f ? c2f + yline : nullptr;
  out[0] = invx * dsum<T, ORDER>(w + g.field + xline, x, g.nx, 1) +
           invy * dsum<T, ORDER>(w + 2 * g.field + yline, y, g.ny, g.nx);
  out[1] = invx * dsum_c2<T, ORDER>(p + xline, c2x, c2c, x, g.nx, 1);
  out[2] = invy * dsum_c2<T, ORDER>(p + yline, c2y, c2c, y, g.ny, g.nx);
  if constexpr (D == 3) {
    const T* c2z = c2f ? c2f + zline : nullptr;
    out[0] += invz * dsum<T, ORDER>(w + 3 * g.field + zline, z, g.nz, plane);
    out[3] = invz * dsum_c2<T, ORDER>(p + zline, c2z, c2c, z, g.nz, plane);
  }
}

template <typename T, int ORDER, int OP>
__device__ __forceinline__ T neg_div(const T* __restrict__ s, int x, int y, int z,
                                     const Geometry& g, T invx, T invy, T invz) {
  const int64_t plane = (int64_t)g.nx * g.ny;
  const int64_t xline = (int64_t)z * plane + (int64_t)y * g.nx;
  const int64_t yline = (int64_t)z * plane + x;
  T d = invx * dsum<T, ORDER>(s + g.field + xline, x, g.nx, 1) +
        invy * dsum<T, ORDER>(s + 2 * g.field + yline, y, g.ny, g.nx);
  if constexpr (OP == OP_AC3D) {
    const int64_t zline = (int64_t)y * g.nx + x;
    d += invz * dsum<T, ORDER>(s + 3 * g.field + zline, z, g.nz, plane);
  }
  return -d;
}

template <typename T>
struct AdjArgs {
  Geometry g;
  const T* c2f;
  T c2c, invx, invy, invz;
  const T* ybar;        // adjoint at the macro step's end (first kernel)
  const T* level;       // forward level y_n (for -div v_n)
  T* P;                 // lambda_{n+1} (final), read at the neighbours
  T* Q;                 // lambda_n (partial), updated in place
  double* yacc;         // sum_j (lambda_0 + lambda_1)
  double* facc;         // sum_j h_j lambda_1
  double* grad;         // dL/dc^2, FP64, [Z][Y][X], or null
  double cw;            // c_j
  double h;             // h_j
  int32_t last;         // this step is n = 1: fold into yacc / facc
  int32_t first_seq;    // the first sequence writes yacc / facc instead of adding
  int32_t nrhs;         // right-hand sides (looped over by each thread)
  int32_t tz;           // adj_tile3d: planes per block (0: the template's TZ)
};

// Step n = N of sequence j: reads w = c_j ybar at the neighbours, writes
// P = lambda_N (final) and Q = lambda_{N-1} (partial, = w/2).
template <typename T, int ORDER, int OP>
__global__ __launch_bounds__(256) void adj_first_kernel(const AdjArgs<T> a) {
  constexpr int F = NFields<OP>::F;
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= a.g.field) return;
  int x, y, z;
  decompose(idx, a.g, x, y, z);
  double gsum = 0.0;
  for (int r = 0; r < a.nrhs; ++r) {
    const int64_t base = (int64_t)r * a.g.state;
    T at[F];
    eval_AT<T, ORDER, OP>(a.ybar + base, a.c2f, a.c2c, x, y, z, a.g, a.invx, a.invy, a.invz, at);
    const T cq = (T)(0.25 * a.cw), ch = (T)(0.5 * a.cw);
    const T h2 = (T)(2.0 * a.h);
    // every load before the first store (the compiler cannot move a load
    // across a store it may alias)
    T yb[F];
#pragma unroll
    for (int q = 0; q < F; ++q) yb[q] = a.ybar[base + q * a.g.field + idx];
    if (a.grad) {
      const T dv = neg_div<T, ORDER, OP>(a.level + base, x, y, z, a.g, a.invx, a.invy, a.invz);
      gsum += 2.0 * a.h * ((double)cq * (double)yb[0]) * (double)dv;
    }
#pragma unroll
    for (int q = 0; q < F; ++q) {
      const int64_t e = base + q * a.g.field + idx;
      a.P[e] = ch * yb[q] + h2 * (cq * at[q]);        // lambda_N
      a.Q[e] = ch * yb[q];                            // lambda_{N-1} so far
    }
  }
  if (a.grad) a.grad[idx] += gsum;
}

// Step n < N: Q += 2h A^T P; gradient from P and y_n; at n = 1 the forward
// Euler transpose is folded in.
template <typename T, int ORDER, int OP>
__global__ __launch_bounds__(256) void adj_lf_kernel(const AdjArgs<T> a) {
  constexpr int F = NFields<OP>::F;
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= a.g.field) return;
  int x, y, z;
  decompose(idx, a.g, x, y, z);
  const T h2 = (T)(2.0 * a.h);
  double gsum = 0.0;
  for (int r = 0; r < a.nrhs; ++r) {
    const int64_t base = (int64_t)r * a.g.state;
    T at[F];
    eval_AT<T, ORDER, OP>(a.P + base, a.c2f, a.c2c, x, y, z, a.g, a.invx, a.invy, a.invz, at);
    // every load before the first store (the compiler cannot move a load
    // across a store it may alias)
    T qo[F], po[F];
    double ya[F], fa[F];
#pragma unroll
    for (int q = 0; q < F; ++q) {
      const int64_t e = base + q * a.g.field + idx;
      qo[q] = a.Q[e];
      po[q] = (a.last || (a.grad && q == 0)) ? a.P[e] : T(0);
      ya[q] = (a.last && !a.first_seq) ? a.yacc[e] : 0.0;
      fa[q] = (a.last && !a.first_seq) ? a.facc[e] : 0.0;
    }
    if (a.grad) {
      const T dv = neg_div<T, ORDER, OP>(a.level + base, x, y, z, a.g, a.invx, a.invy, a.invz);
      gsum += 2.0 * a.h * (double)po[0] * (double)dv;
    }
#pragma unroll
    for (int q = 0; q < F; ++q) {
      const int64_t e = base + q * a.g.field + idx;
      const T qn = qo[q] + h2 * at[q];
      if (!a.last) {
        a.Q[e] = qn;
      } else {
        // here qn = lambda_1 (final) and P = lambda_2 = lambda_0 (its only term)
        const double l1 = (double)qn;
        const double v0 = l1 + (double)po[q];        // lambda_0 + lambda_1
        const double f0 = a.h * l1;                  // h_j lambda_1
        if (a.first_seq) {
          a.yacc[e] = v0;
          a.facc[e] = f0;
        } else {
          a.yacc[e] = ya[q] + v0;
          a.facc[e] = fa[q] + f0;
        }
      }
    }
  }
  if (a.grad) a.grad[idx] += gsum;
}

// dsum_c2 with 32-bit element indices from uniform base pointers (see
// dsum32).
template <typename T, int ORDER>
__device__ __forceinline__ T dsum_c2_32(const T* __restrict__ u, const T* __restrict__ c2f, T c2c,
                                        uint32_t c, int i, int n, uint32_t s) {
  T acc = T(0);
#pragma unroll
  for (int k = 0; k < Fd<ORDER>::R; ++k) {
    const uint32_t iu = c + (uint32_t)(wrap(i + k + 1, n) - i) * s;
    const uint32_t id = c + (uint32_t)(wrap(i - k - 1, n) - i) * s;
    const T up = (c2f ? c2f[iu] : c2c) * u[iu];
    const T dn = (c2f ? c2f[id] : c2c) * u[id];
    acc += Fd<ORDER>::template w<T>(k) * (up - dn);
  }
  return acc;
}

// The two sweeps above for the 3-D operator, marching in z (the layout of
// lf_march3d): each thread walks up its (x, y) column keeping the planes
// z-R..z+R of c^2 u_p, u_vz and the level's v_z in registers, while the x-
// and y-derivatives read the current plane.  FIRST: u = ybar (step n = N),
// else u = P.  The right-hand sides are looped over inside the thread, so
// the c^2 gradient of a point has one writer.  Same products and sums, in
// the same order, as adj_first_kernel / adj_lf_kernel (the gradient adds
// the right-hand sides' terms one at a time).  Fields of fewer than 2^31
// points (32-bit element indices).
template <typename T, int ORDER, int TZ, bool FIRST>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(sizeof(T) == 4 ? 3 : 2)))
void adj_march3d(const AdjArgs<T> a) {
  constexpr int R = Fd<ORDER>::R;
  const int nx = a.g.nx, ny = a.g.ny, nz = a.g.nz;
  const int ntx = (nx + 63) >> 6, nty = (ny + 3) >> 2;
  const int tile = xcd_tile(blockIdx.x, gridDim.x);
  const int tx = tile % ntx;
  const int ty = (tile / ntx) % nty;
  const int tz = tile / (ntx * nty);
  const int x = tx * 64 + (threadIdx.x & 63);
  const int y = ty * 4 + (threadIdx.x >> 6);
  const int z0 = tz * TZ;
  if (x >= nx || y >= ny || z0 >= nz) return;
  const int64_t F1 = a.g.field;
  const uint32_t plane = (uint32_t)nx * (uint32_t)ny;
  const uint32_t pil = (uint32_t)y * (uint32_t)nx + (uint32_t)x;
  const uint32_t snx = (uint32_t)nx;
  const int zend = min(z0 + TZ, nz);
  const bool wantg = a.grad != nullptr;
  const T h2 = (T)(2.0 * a.h);
  const T cq = (T)(0.25 * a.cw), ch = (T)(0.5 * a.cw);
  const T* __restrict__ c2f = a.c2f;
  for (int r = 0; r < a.nrhs; ++r) {
    const int64_t base = (int64_t)r * a.g.state;
    const T* __restrict__ up = (FIRST ? a.ybar : a.P) + base;     // u_p
    const T* __restrict__ ux = up + F1;
    const T* __restrict__ uy = up + 2 * F1;
    const T* __restrict__ uz = up + 3 * F1;
    const T* __restrict__ lx = a.level + base + F1;
    const T* __restrict__ ly = lx + F1;
    const T* __restrict__ lz = ly + F1;
    T qa[2 * R + 1], qb[2 * R + 1], ql[2 * R + 1];
#pragma unroll
    for (int k = 0; k < 2 * R; ++k) {
      const uint32_t e = (uint32_t)wrap(z0 - R + k, nz) * plane + pil;
      qa[k] = (c2f ? c2f[e] : a.c2c) * up[e];
      qb[k] = uz[e];
      ql[k] = wantg ? lz[e] : T(0);
    }
    for (int z = z0; z < zend; ++z) {
      {
        const uint32_t e = (uint32_t)wrap(z + R, nz) * plane + pil;
        qa[2 * R] = (c2f ? c2f[e] : a.c2c) * up[e];
        qb[2 * R] = uz[e];
        ql[2 * R] = wantg ? lz[e] : T(0);
      }
      const uint32_t idx = (uint32_t)z * plane + pil;
      T sb = T(0), sa = T(0);
#pragma unroll
      for (int k = 0; k < R; ++k) {
        sb += Fd<ORDER>::template w<T>(k) * (qb[R + 1 + k] - qb[R - 1 - k]);
        sa += Fd<ORDER>::template w<T>(k) * (qa[R + 1 + k] - qa[R - 1 - k]);
      }
      T at[4];
      at[0] = a.invx * dsum32<T, ORDER>(ux, idx, x, nx, 1) +
              a.invy * dsum32<T, ORDER>(uy, idx, y, ny, snx);
      at[1] = a.invx * dsum_c2_32<T, ORDER>(up, c2f, a.c2c, idx, x, nx, 1);
      at[2] = a.invy * dsum_c2_32<T, ORDER>(up, c2f, a.c2c, idx, y, ny, snx);
      at[0] += a.invz * sb;
      at[3] = a.invz * sa;
      T dv = T(0);
      if (wantg) {
        T sl = T(0);
#pragma unroll
        for (int k = 0; k < R; ++k)
          sl += Fd<ORDER>::template w<T>(k) * (ql[R + 1 + k] - ql[R - 1 - k]);
        T dd = a.invx * dsum32<T, ORDER>(lx, idx, x, nx, 1) +
               a.invy * dsum32<T, ORDER>(ly, idx, y, ny, snx);
        dd += a.invz * sl;
        dv = -dd;
      }
      // every load of the point before its first store (the compiler cannot
      // move a load across a store it may alias)
      const double g0 = wantg ? a.grad[idx] : 0.0;
      if constexpr (FIRST) {
        T yb[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) yb[q] = a.ybar[base + q * F1 + idx];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const int64_t fo = base + q * F1;
          a.P[fo + idx] = ch * yb[q] + h2 * (cq * at[q]);
          a.Q[fo + idx] = ch * yb[q];
        }
        if (wantg) a.grad[idx] = g0 + 2.0 * a.h * ((double)cq * (double)yb[0]) * (double)dv;
      } else {
        T qo[4], po[4];
        double ya[4], fa[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const int64_t fo = base + q * F1;
          qo[q] = a.Q[fo + idx];
          po[q] = (a.last || (wantg && q == 0)) ? a.P[fo + idx] : T(0);
          ya[q] = (a.last && !a.first_seq) ? a.yacc[fo + idx] : 0.0;
          fa[q] = (a.last && !a.first_seq) ? a.facc[fo + idx] : 0.0;
        }
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const int64_t fo = base + q * F1;
          const T qn = qo[q] + h2 * at[q];
          if (!a.last) {
            a.Q[fo + idx] = qn;
          } else {
            const double l1 = (double)qn;
            const double v0 = l1 + (double)po[q];
            const double f0 = a.h * l1;
            if (a.first_seq) {
              a.yacc[fo + idx] = v0;
              a.facc[fo + idx] = f0;
            } else {
              a.yacc[fo + idx] = ya[q] + v0;
              a.facc[fo + idx] = fa[q] + f0;
            }
          }
        }
        if (wantg) a.grad[idx] = g0 + 2.0 * a.h * (double)po[0] * (double)dv;
      }
#pragma unroll
      for (int k = 0; k < 2 * R; ++k) {
        qa[k] = qa[k + 1];
        qb[k] = qb[k + 1];
        ql[k] = ql[k + 1];
      }
    }
  }
}

// The sweeps of adj_march3d in the LDS-tiled layout of lf_tile3d: a block
// of 64 x BY threads covers 64 x BY columns and marches up TZ planes, the
// right-hand sides one after another (so the c^2 gradient of a point keeps
// one writer).  Per plane the block stages c^2 u_p (x and y halo), u_x (x
// halo), u_y (y halo) and, for the gradient (GRAD), the level's v_x (x) and
// v_y (y) in LDS once (two buffers, one barrier per plane); the z-windows
// of c^2 u_p, u_z and the level's v_z stay in registers.  Columns past a
// ragged edge hold the periodic continuation.  Same products and sums, in
// the same order, as adj_march3d.  Fields of fewer than 2^31 points.
template <typename T, int ORDER, int TZ, int BY, bool FIRST, bool GRAD, int WPE>
__global__ __launch_bounds__(64 * BY) __attribute__((amdgpu_waves_per_eu(WPE)))
void adj_tile3d(const AdjArgs<T> a) {
  constexpr int R = Fd<ORDER>::R;
  constexpr int BX = 64, LX = BX + 2 * R, LY = BY + 2 * R, NT = 64 * BY;
  constexpr int NF = GRAD ? 3 : 2;         // staged fields with a y (x) halo
  constexpr int NYP = 2 * R * BX;          // y-halo positions per staged field
  constexpr int NXP = BY * 2 * R;          // x-halo positions per staged field
  constexpr int NYI = (NF * NYP + NT - 1) / NT;   // y-halo items per thread
  static_assert(NF * NXP <= NT, "x halo larger than the block");
  __shared__ T scu[2][LY][LX];             // c^2 u_p
  __shared__ T sux[2][BY][LX];
  __shared__ T suy[2][LY][BX];
  __shared__ T slx[GRAD ? 2 : 1][GRAD ? BY : 1][GRAD ? LX : 1];   // level v_x, v_y
  __shared__ T sly[GRAD ? 2 : 1][GRAD ? LY : 1][GRAD ? BX : 1];
  const uint32_t nx = a.g.nx, ny = a.g.ny;
  const int nz = a.g.nz;
  const int ntx = (int)((nx + BX - 1) / BX), nty = (int)((ny + BY - 1) / BY);
  const int tile = xcd_tile(blockIdx.x, gridDim.x);
  const int tx = tile % ntx, ty = (tile / ntx) % nty, tz = tile / (ntx * nty);
  const int t = threadIdx.x, lx = t & 63, ly = t >> 6;
  const int tzn = a.tz > 0 ? a.tz : TZ;              // planes per block
  const int x0 = tx * BX, y0 = ty * BY, z0 = tz * tzn;
  const int x = x0 + lx, y = y0 + ly;
  const bool valid = x < (int)nx && y < (int)ny;
  const uint32_t F1 = (uint32_t)a.g.field;
  const uint32_t plane = nx * ny;
  const uint32_t own = (uint32_t)pmod(y, ny) * nx + (uint32_t)pmod(x, nx);
  const uint32_t pil = (uint32_t)y * nx + (uint32_t)x;
  const int zend = min(z0 + tzn, nz);
  const T h2 = (T)(2.0 * a.h);
  const T cq = (T)(0.25 * a.cw), ch = (T)(0.5 * a.cw);
  const T* __restrict__ c2f = a.c2f;
  // halo items: y-halo items t + NT i (field 0 c^2 u_p, 1 u_y, 2 level v_y),
  // x-halo item t (field 0 c^2 u_p, 1 u_x, 2 level v_x); position -> column
  auto ycol = [&](int it) {
    const int pos = it % NYP, hr = pos / BX;
    return (uint32_t)pmod(y0 + (hr < R ? hr : BY + hr) - R, ny) * nx +
           (uint32_t)pmod(x0 + pos % BX, nx);
  };
  const bool hx = t < NF * NXP;
  const int xf = t / NXP, xpos = t % NXP, xhc = xpos % (2 * R);
  const int xr = xpos / (2 * R), xc = xhc < R ? xhc : BX + xhc;
  const uint32_t xcol = (uint32_t)pmod(y0 + xr, ny) * nx + (uint32_t)pmod(x0 + xc - R, nx);
  int zb = 0;                              // planes marched so far (buffer parity)
  for (int r = 0; r < a.nrhs; ++r) {
    const int64_t base = (int64_t)r * a.g.state;
    const T* __restrict__ up = (FIRST ? a.ybar : a.P) + base;     // u_p
    const T* __restrict__ ux = up + F1;
    const T* __restrict__ uy = up + 2 * (int64_t)F1;
    const T* __restrict__ uz = up + 3 * (int64_t)F1;
    const T* __restrict__ lvx = a.level + base + F1;
    const T* __restrict__ lvy = lvx + F1;
    const T* __restrict__ lvz = lvy + F1;
    auto cu = [&](uint32_t e) { return (c2f ? c2f[e] : a.c2c) * up[e]; };
    auto yhalo = [&](int it, uint32_t zo) -> T {
      const int f = it / NYP;
      const uint32_t e = zo + ycol(it);
      return f == 0 ? cu(e) : (f == 1 ? uy[e] : lvy[e]);
    };
    auto xhalo = [&](uint32_t zo) -> T {
      const uint32_t e = zo + xcol;
      return xf == 0 ? cu(e) : (xf == 1 ? ux[e] : lvx[e]);
    };
    T qa[2 * R + 1], qb[2 * R + 1], ql[GRAD ? 2 * R + 1 : 1];
#pragma unroll
    for (int k = 0; k <= 2 * R; ++k) {
      const uint32_t e = (uint32_t)pmod(z0 - R + k, nz) * plane + own;
      qa[k] = cu(e);
      qb[k] = uz[e];
      if constexpr (GRAD) ql[k] = lvz[e];
    }
    T oux, ouy, olx = T(0), oly = T(0), hyv[NYI], hxv = T(0);
    {
      const uint32_t zo = (uint32_t)z0 * plane;
      oux = ux[zo + own];
      ouy = uy[zo + own];
      if constexpr (GRAD) {
        olx = lvx[zo + own];
        oly = lvy[zo + own];
      }
#pragma unroll
      for (int i = 0; i < NYI; ++i)
        if (t + NT * i < NF * NYP) hyv[i] = yhalo(t + NT * i, zo);
      if (hx) hxv = xhalo(zo);
    }
    for (int z = z0; z < zend; ++z, ++zb) {
      const int b = zb & 1;
      scu[b][ly + R][lx + R] = qa[R];
      sux[b][ly][lx + R] = oux;
      suy[b][ly + R][lx] = ouy;
      if constexpr (GRAD) {
        slx[b][ly][lx + R] = olx;
        sly[b][ly + R][lx] = oly;
      }
#pragma unroll
      for (int i = 0; i < NYI; ++i) {
        const int it = t + NT * i;
        if (it >= NF * NYP) continue;
        const int f = it / NYP, pos = it % NYP, hr = pos / BX, c = pos % BX;
        const int row = hr < R ? hr : BY + hr;
        if (f == 0) scu[b][row][c + R] = hyv[i];
        else if (f == 1) suy[b][row][c] = hyv[i];
        else if constexpr (GRAD) sly[b][row][c] = hyv[i];
      }
      if (hx) {
        if (xf == 0) scu[b][xr + R][xc] = hxv;
        else if (xf == 1) sux[b][xr][xc] = hxv;
        else if constexpr (GRAD) slx[b][xr][xc] = hxv;
      }
      __syncthreads();
      // the next plane's values, in flight while this plane is evaluated
      T anext = T(0), bnext = T(0), lnext = T(0);
      if (z + 1 < zend) {
        const uint32_t zn = (uint32_t)(z + 1) * plane;
        const uint32_t e = (uint32_t)pmod(z + 1 + R, nz) * plane + own;
        anext = cu(e);
        bnext = uz[e];
        if constexpr (GRAD) lnext = lvz[e];
        oux = ux[zn + own];
        ouy = uy[zn + own];
        if constexpr (GRAD) {
          olx = lvx[zn + own];
          oly = lvy[zn + own];
        }
#pragma unroll
        for (int i = 0; i < NYI; ++i)
          if (t + NT * i < NF * NYP) hyv[i] = yhalo(t + NT * i, zn);
        if (hx) hxv = xhalo(zn);
      }
      T sb = T(0), sa = T(0), dxx = T(0), dyy = T(0), cx = T(0), cy = T(0);
#pragma unroll
      for (int k = 0; k < R; ++k) {
        const T w = Fd<ORDER>::template w<T>(k);
        sb += w * (qb[R + 1 + k] - qb[R - 1 - k]);
        sa += w * (qa[R + 1 + k] - qa[R - 1 - k]);
        dxx += w * (sux[b][ly][lx + R + k + 1] - sux[b][ly][lx + R - k - 1]);
        dyy += w * (suy[b][ly + R + k + 1][lx] - suy[b][ly + R - k - 1][lx]);
        cx += w * (scu[b][ly + R][lx + R + k + 1] - scu[b][ly + R][lx + R - k - 1]);
        cy += w * (scu[b][ly + R + k + 1][lx + R] - scu[b][ly + R - k - 1][lx + R]);
      }
      T at[4];
      at[0] = a.invx * dxx + a.invy * dyy;
      at[1] = a.invx * cx;
      at[2] = a.invy * cy;
      at[0] += a.invz * sb;
      at[3] = a.invz * sa;
      T dv = T(0);
      if constexpr (GRAD) {
        T sl = T(0), gx = T(0), gy = T(0);
#pragma unroll
        for (int k = 0; k < R; ++k) {
          const T w = Fd<ORDER>::template w<T>(k);
          sl += w * (ql[R + 1 + k] - ql[R - 1 - k]);
          gx += w * (slx[b][ly][lx + R + k + 1] - slx[b][ly][lx + R - k - 1]);
          gy += w * (sly[b][ly + R + k + 1][lx] - sly[b][ly + R - k - 1][lx]);
        }
        T dd = a.invx * gx + a.invy * gy;
        dd += a.invz * sl;
        dv = -dd;
      }
      if (valid) {
        // every load of the point is issued before its first store (the
        // compiler cannot move a load across a store it may alias, and loads
        // interleaved with stores would wait for one memory round trip each)
        const uint32_t idx = (uint32_t)z * plane + pil;
        double g0 = 0.0;
        if constexpr (GRAD) g0 = a.grad[idx];
        if constexpr (FIRST) {
          T yb[4];
#pragma unroll
          for (int q = 0; q < 4; ++q) yb[q] = a.ybar[base + q * (int64_t)F1 + idx];
#pragma unroll
          for (int q = 0; q < 4; ++q) {
            const int64_t fo = base + q * (int64_t)F1;
            a.P[fo + idx] = ch * yb[q] + h2 * (cq * at[q]);
            a.Q[fo + idx] = ch * yb[q];
          }
          if constexpr (GRAD) a.grad[idx] = g0 + 2.0 * a.h * ((double)cq * (double)yb[0]) * (double)dv;
        } else {
          T qo[4], po[4];
          double ya[4], fa[4];
#pragma unroll
          for (int q = 0; q < 4; ++q) qo[q] = a.Q[base + q * (int64_t)F1 + idx];
          if (a.last || GRAD) {
#pragma unroll
            for (int q = 0; q < 4; ++q)
              if (a.last || q == 0) po[q] = a.P[base + q * (int64_t)F1 + idx];
          }
          if (a.last && !a.first_seq) {
#pragma unroll
            for (int q = 0; q < 4; ++q) {
              ya[q] = a.yacc[base + q * (int64_t)F1 + idx];
              fa[q] = a.facc[base + q * (int64_t)F1 + idx];
            }
          }
#pragma unroll
          for (int q = 0; q < 4; ++q) {
            const int64_t fo = base + q * (int64_t)F1;
            const T qn = qo[q] + h2 * at[q];
            if (!a.last) {
              a.Q[fo + idx] = qn;
            } else {
              const double l1 = (double)qn;
              const double v0 = l1 + (double)po[q];
              const double f0 = a.h * l1;
              if (a.first_seq) {
                a.yacc[fo + idx] = v0;
                a.facc[fo + idx] = f0;
              } else {
                a.yacc[fo + idx] = ya[q] + v0;
                a.facc[fo + idx] = fa[q] + f0;
              }
            }
          }
          if constexpr (GRAD) a.grad[idx] = g0 + 2.0 * a.h * (double)po[0] * (double)dv;
        }
      }
#pragma unroll
      for (int k = 0; k < 2 * R; ++k) {
        qa[k] = qa[k + 1];
        qb[k] = qb[k + 1];
        if constexpr (GRAD) ql[k] = ql[k + 1];
      }
      qa[2 * R] = anext;
      qb[2 * R] = bnext;
      if constexpr (GRAD) ql[2 * R] = lnext;
    }
  }
}

template <typename T>
struct AdjFinalArgs {
  Geometry g;
  const T* c2f;
  T c2c;
  double invx, invy, invz;
  const double* yacc;
  const double* facc;
  const T* y0;          // forward state at the macro step's start
  T* ybar;              // out: adjoint at the macro step's start
  double* grad;
  int32_t nrhs;
};

// ybar_0 = yacc + A^T facc (FP64), gradient of the shared first evaluation.
template <typename T, int ORDER, int OP>
__global__ __launch_bounds__(256) void adj_final_kernel(const AdjFinalArgs<T> a) {
  constexpr int F = NFields<OP>::F;
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= a.g.field) return;
  int x, y, z;
  decompose(idx, a.g, x, y, z);
  const int64_t plane = (int64_t)a.g.nx * a.g.ny;
  const int64_t xline = (int64_t)z * plane + (int64_t)y * a.g.nx;
  const int64_t yline = (int64_t)z * plane + x;
  const int64_t zline = (int64_t)y * a.g.nx + x;
  auto c2at = [&](int64_t i) { return a.c2f ? (double)a.c2f[i] : (double)a.c2c; };
  double gsum = 0.0;
  for (int r = 0; r < a.nrhs; ++r) {
    const int64_t base = (int64_t)r * a.g.state;
    const double* fp = a.facc + base;
    double at[F];
    at[0] = a.invx * dsum<double, ORDER>(fp + a.g.field + xline, x, a.g.nx, 1) +
            a.invy * dsum<double, ORDER>(fp + 2 * a.g.field + yline, y, a.g.ny, a.g.nx);
    double sx = 0, sy = 0, sz = 0;
#pragma unroll
    for (int k = 0; k < Fd<ORDER>::R; ++k) {
      const int64_t xu = xline + wrap(x + k + 1, a.g.nx), xd = xline + wrap(x - k - 1, a.g.nx);
      const int64_t yu = yline + (int64_t)wrap(y + k + 1, a.g.ny) * a.g.nx;
      const int64_t yd = yline + (int64_t)wrap(y - k - 1, a.g.ny) * a.g.nx;
      const double wk = Fd<ORDER>::template w<double>(k);
      sx += wk * (c2at(xu) * fp[xu] - c2at(xd) * fp[xd]);
      sy += wk * (c2at(yu) * fp[yu] - c2at(yd) * fp[yd]);
      if constexpr (OP == OP_AC3D) {
        const int64_t zu = zline + (int64_t)wrap(z + k + 1, a.g.nz) * plane;
        const int64_t zd = zline + (int64_t)wrap(z - k - 1, a.g.nz) * plane;
        sz += wk * (c2at(zu) * fp[zu] - c2at(zd) * fp[zd]);
      }
    }
    at[1] = a.invx * sx;
    at[2] = a.invy * sy;
    if constexpr (OP == OP_AC3D) {
      at[0] += a.invz * dsum<double, ORDER>(fp + 3 * a.g.field + zline, z, a.g.nz, plane);
      at[3] = a.invz * sz;
    }
    // every load before the first store (the compiler cannot move a load
    // across a store it may alias)
    double ya[F];
#pragma unroll
    for (int q = 0; q < F; ++q) ya[q] = a.yacc[base + q * a.g.field + idx];
    if (a.grad) {
      const T dv = neg_div<T, ORDER, OP>(a.y0 + base, x, y, z, a.g, (T)a.invx, (T)a.invy,
                                         (T)a.invz);
      gsum += fp[idx] * (double)dv;
    }
#pragma unroll
    for (int q = 0; q < F; ++q) a.ybar[base + q * a.g.field + idx] = (T)(ya[q] + at[q]);
  }
  if (a.grad) a.grad[idx] += gsum;
}

// Receivers: traces[r] = p[rhs_r][idx_r] of a state; injection adds
// tbar[r] to the pressure of an adjoint state.
struct RecDesc {
  int64_t idx;
  int32_t rhs;
  int32_t pad;
};

template <typename T>
__global__ void gather_kernel(const T* __restrict__ y, int64_t state, const RecDesc* rec, int n,
                              T* __restrict__ out) {
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= n) return;
  out[r] = y[(int64_t)rec[r].rhs * state + rec[r].idx];
}

// One thread walks the receivers in order, so that receivers sharing a grid
// point add up deterministically; with distinct points (checked on the host)
// every receiver has its own thread.
template <typename T>
__global__ void inject_kernel(T* __restrict__ ybar, int64_t state, const RecDesc* rec, int n,
                              const T* __restrict__ tbar, int distinct) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (distinct) {
    if (t < n) ybar[(int64_t)rec[t].rhs * state + rec[t].idx] += tbar[t];
    return;
  }
  if (t != 0) return;
  for (int r = 0; r < n; ++r) ybar[(int64_t)rec[r].rhs * state + rec[r].idx] += tbar[r];
}

}  // namespace gbs
