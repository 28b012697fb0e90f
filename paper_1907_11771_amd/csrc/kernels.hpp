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
// advection: f_u = -u_x (ORDER = GBS_FD_SPECTRAL: the Fourier derivative).
template <typename T, int ORDER, int OP>
__device__ __forceinline__ void eval_rhs(const T* __restrict__ s, int x, int y, int z,
                                         const Geometry& g, T c2, T invx, T invy, T invz,
                                         T* f) {
  if constexpr (OP == OP_ADV1D) {
    if constexpr (ORDER == GBS_FD_SPECTRAL)
      f[0] = -fourier_dsum<T>(s, x, g.nx, (const T*)g.fourier);
    else
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

// Store that does not keep the line in the caches (the level written now is
// read again only one or two launches later, after the whole grid has
// streamed through).
template <bool NT, typename T>
__device__ __forceinline__ void store(T* p, T v) {
  if constexpr (NT) __builtin_nontemporal_store(v, p);
  else *p = v;
}

// The leap-frog update y_{n+1} = y_{n-1} + 2h f of one point's F fields
// (element offsets e0 + q * fstride) and, in a sequence's last step, the
// average y* with c_j y* added to the FP64 accumulator (or, for the last
// sequence, y_out formed).  `centre(q)` gives the point's value of y_n.
// Every load is issued before the first store: the compiler cannot move a
// load across a store it may alias, so loads interleaved with the stores
// would each wait for a memory round trip.
template <bool NT, int F, typename T, typename Centre>
__device__ __forceinline__ void lf_point(const SeqDesc<T>& d, const StepArgs<T>& a, int64_t e0,
                                         int64_t fstride, const T* f, Centre centre) {
  T o[F];
#pragma unroll
  for (int q = 0; q < F; ++q) o[q] = d.old[e0 + q * fstride];
  if (!(d.mode & MODE_LAST)) {
#pragma unroll
    for (int q = 0; q < F; ++q) store<NT>(d.out + e0 + q * fstride, o[q] + d.h2 * f[q]);
    return;
  }
  T c[F];
  double acc[F];
#pragma unroll
  for (int q = 0; q < F; ++q) {
    c[q] = centre(q);
    acc[q] = (d.mode & MODE_FIRST) ? 0.0 : a.acc[e0 + q * fstride];
  }
#pragma unroll
  for (int q = 0; q < F; ++q) {
    const int64_t e = e0 + q * fstride;
    const T nw = o[q] + d.h2 * f[q];
    const double ys = 0.25 * (((double)o[q] + 2.0 * (double)c[q]) + (double)nw);
    double v = d.cw * ys;
    if (!(d.mode & MODE_FIRST)) v = acc[q] + v;
    if (d.mode & MODE_FINAL) store<NT>(a.yout + e, (T)v);
    else store<NT>(a.acc + e, v);
  }
}

template <typename T, int ORDER, int OP>
__global__ __launch_bounds__(256) void lf_kernel(const StepArgs<T> a) {
  constexpr int F = NFields<OP>::F;
  constexpr int LP = PointLanes<ORDER>::L;
  const int64_t tid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t idx = tid / LP;
  if (idx >= a.g.field) return;          // a point's LP lanes leave together
  const SeqDesc<T>& d = a.seq[blockIdx.y];
  const int64_t rhs = blockIdx.z;
  const int64_t base = rhs * a.g.state;
  int x, y, z;
  decompose(idx, a.g, x, y, z);
  const T c2 = a.c2f ? a.c2f[idx] : a.c2c;
  T f[F];
  if constexpr (LP > 1) {
    f[0] = -fourier_dsum_lanes<T, LP>(d.cur + base, x, a.g.nx, (const T*)a.g.fourier,
                                      (int)(tid % LP));
    if (tid % LP) return;
  } else {
    eval_rhs<T, ORDER, OP>(d.cur + base, x, y, z, a.g, c2, a.invx, a.invy, a.invz, f);
  }
  if (a.g.nsrc) f[0] += source_term<T>(a.src, a.g.nsrc, rhs, idx, d.amp);
  const int64_t e0 = base + idx;
  lf_point<false, F>(d, a, e0, a.g.field, f, [&](int q) { return d.cur[e0 + q * a.g.field]; });
}

// Workgroup index -> tile index so that each of the 8 XCDs (which receive
// workgroups round-robin) works on one contiguous band of tiles, keeping the
// stencil's neighbour rows in the same L2.
__device__ __forceinline__ int xcd_tile(int b, int nblocks) {
  if (nblocks % 8) return b;
  return (b % 8) * (nblocks / 8) + b / 8;
}

// 2-D acoustic leap-frog sweep, marching in y: a 256-thread block covers 64
// columns x 4 strips of TY rows; every thread walks down its column keeping
// the rows y-R..y+R of p and v_y in registers (the y-derivatives), while the
// x-derivatives read the current row (cache-resident across the wavefront).
// Same arithmetic, in the same order, as lf_kernel.
template <typename T, int ORDER, int TY, bool NT>
__global__ __launch_bounds__(256) void lf_march2d(const StepArgs<T> a) {
  constexpr int R = Fd<ORDER>::R;
  const int nx = a.g.nx, ny = a.g.ny;
  const int ntx = (nx + 63) >> 6;
  const int tile = xcd_tile(blockIdx.x, gridDim.x);
  const int tx = tile % ntx, ty = tile / ntx;
  const int x = tx * 64 + (threadIdx.x & 63);
  const int y0 = ty * 4 * TY + (threadIdx.x >> 6) * TY;
  if (x >= nx || y0 >= ny) return;
  const SeqDesc<T>& d = a.seq[blockIdx.y];
  const int64_t rhs = blockIdx.z;
  const int64_t base = rhs * a.g.state;
  const int64_t F1 = a.g.field, F2 = 2 * a.g.field;
  const T* __restrict__ cp = d.cur + base;
  const T* __restrict__ cvx = cp + F1;
  const T* __restrict__ cvy = cp + F2;
  T pw[2 * R + 1], vw[2 * R + 1];
#pragma unroll
  for (int k = 0; k < 2 * R; ++k) {
    const int64_t row = (int64_t)wrap(y0 - R + k, ny) * nx + x;
    pw[k] = cp[row];
    vw[k] = cvy[row];
  }
#pragma unroll
  for (int i = 0; i < TY; ++i) {
    const int y = y0 + i;
    if (y >= ny) break;
    {
      const int64_t row = (int64_t)wrap(y + R, ny) * nx + x;
      pw[2 * R] = cp[row];
      vw[2 * R] = cvy[row];
    }
    const int64_t rowoff = (int64_t)y * nx;
    T syp = T(0), syv = T(0);
#pragma unroll
    for (int k = 0; k < R; ++k) {
      syp += Fd<ORDER>::template w<T>(k) * (pw[R + 1 + k] - pw[R - 1 - k]);
      syv += Fd<ORDER>::template w<T>(k) * (vw[R + 1 + k] - vw[R - 1 - k]);
    }
    const T sxp = dsum<T, ORDER>(cp + rowoff, x, nx, 1);
    const T sxv = dsum<T, ORDER>(cvx + rowoff, x, nx, 1);
    const T c2 = a.c2f ? a.c2f[rowoff + x] : a.c2c;
    const T dvx = a.invx * sxv;
    const T dvy = a.invy * syv;
    T f[3];
    f[0] = -(c2 * (dvx + dvy));
    f[1] = -(a.invx * sxp);
    f[2] = -(a.invy * syp);
    const int64_t idx = rowoff + x;
    if (a.g.nsrc) f[0] += source_term<T>(a.src, a.g.nsrc, rhs, idx, d.amp);
    lf_point<NT, 3>(d, a, base + idx, F1, f,
                    [&](int q) { return q == 0 ? pw[R] : (q == 1 ? cvx[idx] : vw[R]); });
#pragma unroll
    for (int k = 0; k < 2 * R; ++k) {
      pw[k] = pw[k + 1];
      vw[k] = vw[k + 1];
    }
  }
}

// 3-D acoustic leap-frog sweep, marching in z: a 256-thread block covers
// 64 columns x 4 rows of one z-chunk of TZ planes; every thread walks up its
// (x, y) column keeping the planes z-R..z+R of p and v_z in registers (the
// z-derivatives), while the x- and y-derivatives read the current plane
// (its rows are shared by the neighbouring blocks, which march in step).
// Same arithmetic, in the same order, as lf_kernel.  (64-bit addressing:
// measured faster here than 32-bit offsets, which raise the occupancy and
// with it the L2 working set.)
template <typename T, int ORDER, int TZ, bool NT>
__global__ __launch_bounds__(256) void lf_march3d(const StepArgs<T> a) {
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
  const SeqDesc<T>& d = a.seq[blockIdx.y];
  const int64_t rhs = blockIdx.z;
  const int64_t base = rhs * a.g.state;
  const int64_t F1 = a.g.field, F2 = 2 * a.g.field, F3 = 3 * a.g.field;
  const int64_t plane = (int64_t)nx * ny;
  const int64_t pil = (int64_t)y * nx + x;
  const T* __restrict__ cp = d.cur + base;
  const T* __restrict__ cvx = cp + F1;
  const T* __restrict__ cvy = cp + F2;
  const T* __restrict__ cvz = cp + F3;
  T pw[2 * R + 1], vw[2 * R + 1];
#pragma unroll
  for (int k = 0; k < 2 * R; ++k) {
    const int64_t e = (int64_t)wrap(z0 - R + k, nz) * plane + pil;
    pw[k] = cp[e];
    vw[k] = cvz[e];
  }
  const int zend = min(z0 + TZ, nz);
  // the plane z + R that step z needs is loaded one step ahead, so that its
  // latency overlaps the previous step's work
  {
    const int64_t e = (int64_t)wrap(z0 + R, nz) * plane + pil;
    pw[2 * R] = cp[e];
    vw[2 * R] = cvz[e];
  }
  for (int z = z0; z < zend; ++z) {
    T pnext = T(0), vnext = T(0);
    if (z + 1 < zend) {
      const int64_t e = (int64_t)wrap(z + 1 + R, nz) * plane + pil;
      pnext = cp[e];
      vnext = cvz[e];
    }
    const int64_t zoff = (int64_t)z * plane;
    const int64_t row = zoff + (int64_t)y * nx;
    const int64_t col = zoff + x;
    T szp = T(0), szv = T(0);
#pragma unroll
    for (int k = 0; k < R; ++k) {
      szp += Fd<ORDER>::template w<T>(k) * (pw[R + 1 + k] - pw[R - 1 - k]);
      szv += Fd<ORDER>::template w<T>(k) * (vw[R + 1 + k] - vw[R - 1 - k]);
    }
    const int64_t idx = zoff + pil;
    const T c2 = a.c2f ? a.c2f[idx] : a.c2c;
    const T dvx = a.invx * dsum<T, ORDER>(cvx + row, x, nx, 1);
    const T dvy = a.invy * dsum<T, ORDER>(cvy + col, y, ny, nx);
    const T dvz = a.invz * szv;
    T f[4];
    f[0] = -(c2 * ((dvx + dvy) + dvz));
    f[1] = -(a.invx * dsum<T, ORDER>(cp + row, x, nx, 1));
    f[2] = -(a.invy * dsum<T, ORDER>(cp + col, y, ny, nx));
    f[3] = -(a.invz * szp);
    if (a.g.nsrc) f[0] += source_term<T>(a.src, a.g.nsrc, rhs, idx, d.amp);
    lf_point<NT, 4>(d, a, base + idx, F1, f, [&](int q) {
      return q == 0 ? pw[R] : (q == 3 ? vw[R] : (q == 1 ? cvx[idx] : cvy[idx]));
    });
#pragma unroll
    for (int k = 0; k < 2 * R; ++k) {
      pw[k] = pw[k + 1];
      vw[k] = vw[k + 1];
    }
    pw[2 * R] = pnext;
    vw[2 * R] = vnext;
  }
}

// 3-D acoustic sweeps with the x/y neighbourhood of every plane staged in
// LDS.  A 1024-thread block covers a 64 x 16 tile of (x, y) columns and
// marches up tzn planes; every thread keeps the planes z-R..z+R of p and v_z
// of its column in registers (the z-derivatives).  Per plane the block
// writes p, v_x and v_y of its tile, with the R-wide halo of p and v_x along
// x and of p and v_y along y, to LDS once (two buffers, one barrier per
// plane), and the x- and y-derivatives read LDS: a value of the plane is
// fetched from L2/HBM once per block that needs it (1.25 halo values per
// tile point) instead of once per thread that needs it.  Columns and rows
// past a ragged edge hold the periodic continuation, so every valid column
// sees its true neighbours.  Same stencil sums, in the same order, as
// eval_rhs.  `point(idx, dvx, dvy, dvz, f, c)` receives, for every valid
// column, the flat index, the velocity derivatives, f_v (f[1..3]) and the
// plane's four values.  (Loading the point's other inputs a plane ahead
// needs registers that make the sweep spill.)
template <typename T, int ORDER, typename Point>
__device__ __forceinline__ void tile3d_march(const T* __restrict__ cp, const Geometry& g,
                                             T invx, T invy, T invz, const int tile,
                                             const int tzn, Point point) {
  constexpr int R = Fd<ORDER>::R;
  constexpr int BX = 64, BY = 16, LX = BX + 2 * R, LY = BY + 2 * R;
  constexpr int NYH = 2 * R * BX * 2;          // y-halo values (p, v_y) per plane
  constexpr int NXH = BY * 2 * R * 2;          // x-halo values (p, v_x) per plane
  static_assert(NYH <= 1024 && NXH <= 1024, "halo larger than the block");
  __shared__ T sp[2][LY][LX];
  __shared__ T svx[2][BY][LX];
  __shared__ T svy[2][LY][BX];
  const int nx = g.nx, ny = g.ny, nz = g.nz;
  const int ntx = (nx + BX - 1) / BX, nty = (ny + BY - 1) / BY;
  const int tx = tile % ntx, ty = (tile / ntx) % nty, tz = tile / (ntx * nty);
  const int t = threadIdx.x, lx = t & 63, ly = t >> 6;
  const int x0 = tx * BX, y0 = ty * BY, z0 = tz * tzn;
  const int x = x0 + lx, y = y0 + ly;
  const bool valid = x < nx && y < ny;
  const int64_t F1 = g.field;
  const int64_t plane = (int64_t)nx * ny;
  const int64_t own = (int64_t)pmod(y, ny) * nx + pmod(x, nx);   // column within a plane
  const T* __restrict__ cvx = cp + F1;
  const T* __restrict__ cvy = cp + 2 * F1;
  const T* __restrict__ cvz = cp + 3 * F1;
  // this thread's halo values: one of the y-halo (field yf, LDS row yr, column
  // yc) and, for the first NXH threads, one of the x-halo
  const bool hy = t < NYH, hx = t < NXH;
  int yr = 0, yc = 0, xr = 0, xc = 0;
  int64_t ycol = 0, xcol = 0;
  const T* ysrc = cp;
  const T* xsrc = cp;
  if (hy) {
    const int f = t / (2 * R * BX), pos = t % (2 * R * BX), hr = pos / BX;
    yc = pos % BX;
    yr = hr < R ? hr : BY + hr;                               // LDS row (0..R-1, BY+R..)
    ycol = (int64_t)pmod(y0 + yr - R, ny) * nx + pmod(x0 + yc, nx);
    ysrc = f == 0 ? cp : cvy;
  }
  if (hx) {
    const int f = t / (BY * 2 * R), pos = t % (BY * 2 * R), hc = pos % (2 * R);
    xr = pos / (2 * R);
    xc = hc < R ? hc : BX + hc;                               // LDS column
    xcol = (int64_t)pmod(y0 + xr, ny) * nx + pmod(x0 + xc - R, nx);
    xsrc = f == 0 ? cp : cvx;
  }
  const bool yp = hy && t < NYH / 2, xp = hx && t < NXH / 2;  // halo of p (else v_y / v_x)
  T pw[2 * R + 1], vw[2 * R + 1];
#pragma unroll
  for (int k = 0; k <= 2 * R; ++k) {
    const int64_t e = (int64_t)pmod(z0 - R + k, nz) * plane + own;
    pw[k] = cp[e];
    vw[k] = cvz[e];
  }
  const int zend = min(z0 + tzn, nz);
  const int64_t pil = (int64_t)y * nx + x;         // valid columns only
  T vxo, vyo, hyv = T(0), hxv = T(0);
  {
    const int64_t zo = (int64_t)z0 * plane;
    vxo = cvx[zo + own];
    vyo = cvy[zo + own];
    if (hy) hyv = ysrc[zo + ycol];
    if (hx) hxv = xsrc[zo + xcol];
  }
  for (int z = z0; z < zend; ++z) {
    const int b = z & 1;
    sp[b][ly + R][lx + R] = pw[R];
    svx[b][ly][lx + R] = vxo;
    svy[b][ly + R][lx] = vyo;
    if (hy) {
      if (yp) sp[b][yr][yc + R] = hyv;
      else svy[b][yr][yc] = hyv;
    }
    if (hx) {
      if (xp) sp[b][xr + R][xc] = hxv;
      else svx[b][xr][xc] = hxv;
    }
    const T cvxc = vxo, cvyc = vyo;
    __syncthreads();
    // the next plane's stencil values, in flight while this plane is evaluated
    T pnext = T(0), vnext = T(0);
    if (z + 1 < zend) {
      const int64_t zn = (int64_t)(z + 1) * plane;
      const int64_t e = (int64_t)pmod(z + 1 + R, nz) * plane + own;
      pnext = cp[e];
      vnext = cvz[e];
      vxo = cvx[zn + own];
      vyo = cvy[zn + own];
      if (hy) hyv = ysrc[zn + ycol];
      if (hx) hxv = xsrc[zn + xcol];
    }
    T sxp = T(0), syp = T(0), sxv = T(0), syv = T(0), szp = T(0), szv = T(0);
#pragma unroll
    for (int k = 0; k < R; ++k) {
      const T w = Fd<ORDER>::template w<T>(k);
      sxv += w * (svx[b][ly][lx + R + k + 1] - svx[b][ly][lx + R - k - 1]);
      syv += w * (svy[b][ly + R + k + 1][lx] - svy[b][ly + R - k - 1][lx]);
      sxp += w * (sp[b][ly + R][lx + R + k + 1] - sp[b][ly + R][lx + R - k - 1]);
      syp += w * (sp[b][ly + R + k + 1][lx + R] - sp[b][ly + R - k - 1][lx + R]);
      szp += w * (pw[R + 1 + k] - pw[R - 1 - k]);
      szv += w * (vw[R + 1 + k] - vw[R - 1 - k]);
    }
    if (valid) {
      const T dvx = invx * sxv;
      const T dvy = invy * syv;
      const T dvz = invz * szv;
      T f[4], c[4] = {pw[R], cvxc, cvyc, vw[R]};
      f[1] = -(invx * sxp);
      f[2] = -(invy * syp);
      f[3] = -(invz * szp);
      point((int64_t)z * plane + pil, dvx, dvy, dvz, f, c);
    }
#pragma unroll
    for (int k = 0; k < 2 * R; ++k) {
      pw[k] = pw[k + 1];
      vw[k] = vw[k + 1];
    }
    pw[2 * R] = pnext;
    vw[2 * R] = vnext;
  }
}

// One 1024-thread block per CU (4 waves per SIMD, up to 128 VGPRs) in both
// precisions.  Two blocks per CU would need the FP32 sweep in 64 VGPRs, where
// it spills, and each reload from the spill area waits for the plane's
// prefetched loads as well; with a point's loads issued ahead of its stores
// one block keeps enough memory operations in flight.
template <typename T>
constexpr int tile3d_waves() { return 4; }

// Tiles of the 64 x 16 x tzn blocking of lf_tile3d / first_tile3d.
__device__ __forceinline__ int tile3d_count(const Geometry& g, int tzn) {
  return ((g.nx + 63) / 64) * ((g.ny + 15) / 16) * ((g.nz + tzn - 1) / tzn);
}

// Whether a point source of right-hand side `rhs` lies in tile `tile` of
// that blocking (its 64 x 16 columns and tzn planes, as tile3d_march lays
// them out).  Found once per block, so that the sweeps search the sources
// per point only in the few blocks that hold one.
__device__ __forceinline__ bool tile3d_has_source(const SrcDesc* src, int nsrc, int64_t rhs,
                                                  const Geometry& g, int tile, int tzn) {
  const int ntx = (g.nx + 63) / 64, nty = (g.ny + 15) / 16;
  const int x0 = (tile % ntx) * 64, y0 = ((tile / ntx) % nty) * 16;
  const int z0 = (tile / (ntx * nty)) * tzn, z1 = min(z0 + tzn, g.nz);
  for (int k = 0; k < nsrc; ++k) {
    if (src[k].rhs != rhs) continue;
    int x, y, z;
    decompose(src[k].idx, g, x, y, z);
    if (x >= x0 && x < x0 + 64 && y >= y0 && y < y0 + 16 && z >= z0 && z < z1) return true;
  }
  return false;
}

// Workgroup index -> (tile, sequence) for a launch of n sequences over
// `tiles` tiles: the n workgroups of one tile are consecutive on one XCD
// (they read the same c^2 tile, which then comes from that XCD's L2), and
// each XCD works on one contiguous band of tiles as in xcd_tile.
__device__ __forceinline__ void xcd_tile_seq(int b, int tiles, int n, int& tile, int& seq) {
  if (tiles % 8) {
    tile = b / n;
    seq = b % n;
    return;
  }
  const int i = b / 8;
  tile = (b % 8) * (tiles / 8) + i / n;
  seq = i % n;
}

template <typename T, int ORDER, int TZ>
__global__ __launch_bounds__(1024) __attribute__((amdgpu_waves_per_eu(tile3d_waves<T>())))
void lf_tile3d(const StepArgs<T> a) {
  const int tzn = a.tz > 0 ? a.tz : TZ;
  const int tiles = tile3d_count(a.g, tzn);
  int tile, sq;
  xcd_tile_seq(blockIdx.x, tiles, gridDim.x / tiles, tile, sq);
  const SeqDesc<T>& d = a.seq[sq];
  const int64_t rhs = blockIdx.z;
  const int64_t base = rhs * a.g.state;
  const int64_t F1 = a.g.field;
  const bool srcs = a.g.nsrc && tile3d_has_source(a.src, a.g.nsrc, rhs, a.g, tile, tzn);
  tile3d_march<T, ORDER>(
      d.cur + base, a.g, a.invx, a.invy, a.invz, tile, tzn,
      [&](int64_t idx, T dvx, T dvy, T dvz, T* f, const T* c) {
        // every load of the point is issued before its first store: the
        // compiler cannot move a load across a store it may alias, and loads
        // interleaved with stores would wait for one memory round trip each
        T c2 = a.c2c;
        if (a.c2f) c2 = a.c2f[idx];
        T o[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) o[q] = d.old[base + q * F1 + idx];
        f[0] = -(c2 * ((dvx + dvy) + dvz));
        if (srcs) f[0] += source_term<T>(a.src, a.g.nsrc, rhs, idx, d.amp);
        if (!(d.mode & MODE_LAST)) {
#pragma unroll
          for (int q = 0; q < 4; ++q)
            // read back only by the next launch, after the whole grid
            __builtin_nontemporal_store(o[q] + d.h2 * f[q], d.out + base + q * F1 + idx);
          return;
        }
        double acc[4] = {0.0, 0.0, 0.0, 0.0};
        if (!(d.mode & MODE_FIRST)) {
#pragma unroll
          for (int q = 0; q < 4; ++q) acc[q] = a.acc[base + q * F1 + idx];
        }
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const int64_t e = base + q * F1 + idx;
          const T nw = o[q] + d.h2 * f[q];
          const double ys = 0.25 * (((double)o[q] + 2.0 * (double)c[q]) + (double)nw);
          double v = d.cw * ys;
          if (!(d.mode & MODE_FIRST)) v = acc[q] + v;
          if (d.mode & MODE_FINAL) a.yout[e] = (T)v;
          else a.acc[e] = v;
        }
      });
}

// The shared first evaluation and the forward-Euler steps of every
// sequence in the LDS-tiled layout of lf_tile3d.
template <typename T, int ORDER, int TZ>
__global__ __launch_bounds__(1024) __attribute__((amdgpu_waves_per_eu(tile3d_waves<T>())))
void first_tile3d(const FirstArgs<T> a) {
  const int64_t rhs = blockIdx.z;
  const int64_t base = rhs * a.g.state;
  const int64_t F1 = a.g.field;
  const int tile = xcd_tile(blockIdx.x, gridDim.x), tzn = a.tz > 0 ? a.tz : TZ;
  const bool srcs = a.g.nsrc && tile3d_has_source(a.src, a.g.nsrc, rhs, a.g, tile, tzn);
  tile3d_march<T, ORDER>(
      a.y0 + base, a.g, a.invx, a.invy, a.invz, tile, tzn,
      [&](int64_t idx, T dvx, T dvy, T dvz, T* f, const T* c) {
        const T c2 = a.c2f ? a.c2f[idx] : a.c2c;
        f[0] = -(c2 * ((dvx + dvy) + dvz));
        if (srcs) f[0] += source_term<T>(a.src, a.g.nsrc, rhs, idx, a.amp);
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const int64_t fo = base + q * F1;
          for (int j = 0; j < a.nseq; ++j)
            __builtin_nontemporal_store(c[q] + a.h[j] * f[q], a.out[j] + fo + idx);
        }
      });
}

// The shared first evaluation and the forward-Euler steps of every
// sequence, 3-D, in the z-marching layout of lf_march3d.  Same arithmetic,
// in the same order, as first_kernel.
template <typename T, int ORDER, int TZ>
__global__ __launch_bounds__(256) void first_march3d(const FirstArgs<T> a) {
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
  const int64_t rhs = blockIdx.z;
  const int64_t base = rhs * a.g.state;
  const int64_t F1 = a.g.field;
  const uint32_t plane = (uint32_t)nx * (uint32_t)ny;
  const uint32_t pil = (uint32_t)y * (uint32_t)nx + (uint32_t)x;
  const T* __restrict__ cp = a.y0 + base;
  const T* __restrict__ cvx = cp + F1;
  const T* __restrict__ cvy = cp + 2 * F1;
  const T* __restrict__ cvz = cp + 3 * F1;
  T pw[2 * R + 1], vw[2 * R + 1];
#pragma unroll
  for (int k = 0; k < 2 * R; ++k) {
    const uint32_t e = (uint32_t)wrap(z0 - R + k, nz) * plane + pil;
    pw[k] = cp[e];
    vw[k] = cvz[e];
  }
  const int zend = min(z0 + TZ, nz);
  for (int z = z0; z < zend; ++z) {
    {
      const uint32_t e = (uint32_t)wrap(z + R, nz) * plane + pil;
      pw[2 * R] = cp[e];
      vw[2 * R] = cvz[e];
    }
    const uint32_t idx = (uint32_t)z * plane + pil;
    T szp = T(0), szv = T(0);
#pragma unroll
    for (int k = 0; k < R; ++k) {
      szp += Fd<ORDER>::template w<T>(k) * (pw[R + 1 + k] - pw[R - 1 - k]);
      szv += Fd<ORDER>::template w<T>(k) * (vw[R + 1 + k] - vw[R - 1 - k]);
    }
    const T c2 = a.c2f ? a.c2f[idx] : a.c2c;
    const T dvx = a.invx * dsum32<T, ORDER>(cvx, idx, x, nx, 1);
    const T dvy = a.invy * dsum32<T, ORDER>(cvy, idx, y, ny, (uint32_t)nx);
    const T dvz = a.invz * szv;
    T f[4];
    f[0] = -(c2 * ((dvx + dvy) + dvz));
    f[1] = -(a.invx * dsum32<T, ORDER>(cp, idx, x, nx, 1));
    f[2] = -(a.invy * dsum32<T, ORDER>(cp, idx, y, ny, (uint32_t)nx));
    f[3] = -(a.invz * szp);
    if (a.g.nsrc) f[0] += source_term<T>(a.src, a.g.nsrc, rhs, idx, a.amp);
    const T v0[4] = {pw[R], cvx[idx], cvy[idx], vw[R]};
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int64_t fo = base + q * F1;
      for (int j = 0; j < a.nseq; ++j) a.out[j][fo + idx] = v0[q] + a.h[j] * f[q];
    }
#pragma unroll
    for (int k = 0; k < 2 * R; ++k) {
      pw[k] = pw[k + 1];
      vw[k] = vw[k + 1];
    }
  }
}

template <typename T, int ORDER, int OP>
__global__ __launch_bounds__(256) void first_kernel(const FirstArgs<T> a) {
  constexpr int F = NFields<OP>::F;
  constexpr int LP = PointLanes<ORDER>::L;
  const int64_t tid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t idx = tid / LP;
  if (idx >= a.g.field) return;
  const int64_t rhs = blockIdx.z;
  const int64_t base = rhs * a.g.state;
  int x, y, z;
  decompose(idx, a.g, x, y, z);
  const T c2 = a.c2f ? a.c2f[idx] : a.c2c;
  T f[F];
  if constexpr (LP > 1) {
    f[0] = -fourier_dsum_lanes<T, LP>(a.y0 + base, x, a.g.nx, (const T*)a.g.fourier,
                                      (int)(tid % LP));
    if (tid % LP) return;
  } else {
    eval_rhs<T, ORDER, OP>(a.y0 + base, x, y, z, a.g, c2, a.invx, a.invy, a.invz, f);
  }
  if (a.g.nsrc) f[0] += source_term<T>(a.src, a.g.nsrc, rhs, idx, a.amp);
#pragma unroll
  for (int q = 0; q < F; ++q) {
    const int64_t e = base + q * a.g.field + idx;
    const T v0 = a.y0[e];
    for (int j = 0; j < a.nseq; ++j) a.out[j][e] = v0 + a.h[j] * f[q];
  }
}

// Classical RK4 on the same operators (the comparison method of Sect. 3.8
// and App. A), one launch per stage, every point independent:
//   stage 0: K = k1,       next = y + h/2 k1
//   stage 1: K += 2 k2,    next = y + h/2 k2
//   stage 2: K += 2 k3,    next = y + h k3
//   stage 3: y_new = y + h/6 (K + k4)
// with k_s = f(t_s, stage input).  K is kept in FP64 (FP32 stepping keeps
// the stage inputs in FP32, as the extrapolated step keeps its levels).
template <typename T>
struct RK4Args {
  Geometry g;
  SrcDesc src[GBS_MAX_SRC];
  const T* c2f;
  T c2c, invx, invy, invz;
  const T* yn;       // the state at the step's start
  const T* ys;       // this stage's input
  T* out;            // next stage's input, or the new state (stage 3)
  double* acc;       // K (FP64, state-sized)
  double h;
  double amp;        // source wavelet at this stage's time
  int32_t stage;
};

template <typename T, int ORDER, int OP>
__global__ __launch_bounds__(256) void rk4_stage(const RK4Args<T> a) {
  constexpr int F = NFields<OP>::F;
  constexpr int LP = PointLanes<ORDER>::L;
  const int64_t tid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t idx = tid / LP;
  if (idx >= a.g.field) return;
  const int64_t rhs = blockIdx.z;
  const int64_t base = rhs * a.g.state;
  int x, y, z;
  decompose(idx, a.g, x, y, z);
  const T c2 = a.c2f ? a.c2f[idx] : a.c2c;
  T f[F];
  if constexpr (LP > 1) {
    f[0] = -fourier_dsum_lanes<T, LP>(a.ys + base, x, a.g.nx, (const T*)a.g.fourier,
                                      (int)(tid % LP));
    if (tid % LP) return;
  } else {
    eval_rhs<T, ORDER, OP>(a.ys + base, x, y, z, a.g, c2, a.invx, a.invy, a.invz, f);
  }
  if (a.g.nsrc) f[0] += source_term<T>(a.src, a.g.nsrc, rhs, idx, a.amp);
  // every load of the point before its first store (the compiler cannot move
  // a load across a store it may alias)
  T yn[F];
  double acc[F];
#pragma unroll
  for (int q = 0; q < F; ++q) {
    const int64_t e = base + q * a.g.field + idx;
    yn[q] = a.yn[e];
    acc[q] = a.stage == 0 ? 0.0 : a.acc[e];
  }
#pragma unroll
  for (int q = 0; q < F; ++q) {
    const int64_t e = base + q * a.g.field + idx;
    const double k = (double)f[q];
    if (a.stage == 0) {
      a.acc[e] = k;
      a.out[e] = yn[q] + (T)(0.5 * a.h) * f[q];
    } else if (a.stage < 3) {
      a.acc[e] = acc[q] + 2.0 * k;
      a.out[e] = yn[q] + (T)(a.stage == 1 ? 0.5 * a.h : a.h) * f[q];
    } else {
      a.out[e] = (T)((double)yn[q] + (a.h / 6.0) * (acc[q] + k));
    }
  }
}

}  // namespace gbs
