// Device-side building blocks: periodic centred first-derivative stencils
// of order 4 and 8, and the per-launch argument blocks of the step kernels.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "../../include/gbs.h"

namespace gbs {

// D u_i = (1/dx) sum_{k=1..R} a_k (u_{i+k} - u_{i-k}); the a_k are written
// as integers W_k over a common denominator DEN, so that
// D u_i = inv * sum_k W_k (u_{i+k} - u_{i-k}) with inv = n / DEN.
template <int ORDER>
struct Fd;
template <>
struct Fd<4> {
  static constexpr int R = 2;
  static constexpr double DEN = 12.0;
  template <typename T>
  __device__ static T w(int k) { return k == 0 ? T(8) : T(-1); }
};
template <>
struct Fd<8> {
  static constexpr int R = 4;
  static constexpr double DEN = 840.0;
  template <typename T>
  __device__ static T w(int k) {
    return k == 0 ? T(672) : (k == 1 ? T(-168) : (k == 2 ? T(32) : T(-3)));
  }
};

__device__ __forceinline__ int wrap(int i, int n) { return i < 0 ? i + n : (i >= n ? i - n : i); }

// a mod n in [0, n) for any int a (n > 0)
__device__ __forceinline__ int pmod(int a, int n) {
  int r = a % n;
  return r < 0 ? r + n : r;
}

// Sum_k W_k (u[i+k] - u[i-k]) along an axis with stride `stride` and
// periodic length n, around the index `i` (0 <= i < n); `base` points at
// element 0 of that line.
template <typename T, int ORDER>
__device__ __forceinline__ T dsum(const T* __restrict__ base, int i, int n, int64_t stride) {
  T s = T(0);
#pragma unroll
  for (int k = 0; k < Fd<ORDER>::R; ++k) {
    const T up = base[(int64_t)wrap(i + k + 1, n) * stride];
    const T dn = base[(int64_t)wrap(i - k - 1, n) * stride];
    s += Fd<ORDER>::template w<T>(k) * (up - dn);
  }
  return s;
}

// dsum for a field addressed by 32-bit element indices from a uniform base
// pointer (fields of fewer than 2^31 points): c is the centre's index, i its
// coordinate along the axis (period n), s the axis stride.  Same products
// and sums, in the same order, as dsum; the narrow offsets let loads use a
// scalar base and one 32-bit register per address.
template <typename T, int ORDER>
__device__ __forceinline__ T dsum32(const T* __restrict__ f, uint32_t c, int i, int n,
                                    uint32_t s) {
  T acc = T(0);
#pragma unroll
  for (int k = 0; k < Fd<ORDER>::R; ++k) {
    const uint32_t up = c + (uint32_t)(wrap(i + k + 1, n) - i) * s;
    const uint32_t dn = c + (uint32_t)(wrap(i - k - 1, n) - i) * s;
    acc += Fd<ORDER>::template w<T>(k) * (f[up] - f[dn]);
  }
  return acc;
}

// Fourier derivative on n points of [0,1) written as a centred difference
// over the whole period: D u_i = sum_{k=1..K} b_k (u[i+k] - u[i-k]), K =
// (n-1)/2, b_k = pi (-1)^(k+1) cot(pi k / n) for even n (the mode n/2 drops
// out: cot(pi/2) = 0) and pi (-1)^(k+1) / sin(pi k / n) for odd n; `b` holds
// b_1..b_K.  Pairing u[i+k] with u[i-k] keeps the large weights of small k
// on differences of nearby values.  The K terms are summed with Kahan's
// compensation: a plain running sum of this many terms loses about sqrt(K)
// ulps on grid-scale data (8e-15 relative at n = 8192, against 4e-16 for an
// FFT), the compensated one stays near one ulp.
template <typename T>
__device__ __forceinline__ T fourier_dsum(const T* __restrict__ u, int i, int n,
                                          const T* __restrict__ b) {
  const int K = (n - 1) / 2;
  T sum = T(0), comp = T(0);
  // unrolled so that the loads of several k are in flight at once (the
  // compensated sum itself is a dependent chain)
#pragma unroll 8
  for (int k = 1; k <= K; ++k) {
    const int up = i + k < n ? i + k : i + k - n;
    const int dn = i - k >= 0 ? i - k : i - k + n;
    const T y = b[k - 1] * (u[up] - u[dn]) - comp;
    const T t = sum + y;
    comp = (t - sum) - y;
    sum = t;
  }
  return sum;
}

// The same sum split over L consecutive lanes (L a power of two dividing 64):
// lane `sub` of the point takes k = 1 + sub, 1 + sub + L, ... with its own
// compensated sum, and a butterfly over the L lanes adds the partial sums
// and their compensations (every lane ends with the same value: each
// pairwise addition is commutative).  The point's L lanes must all be
// active.
template <typename T, int L>
__device__ __forceinline__ T fourier_dsum_lanes(const T* __restrict__ u, int i, int n,
                                                const T* __restrict__ b, int sub) {
  const int K = (n - 1) / 2;
  T sum = T(0), comp = T(0);
#pragma unroll 4
  for (int k = 1 + sub; k <= K; k += L) {
    const int up = i + k < n ? i + k : i + k - n;
    const int dn = i - k >= 0 ? i - k : i - k + n;
    const T y = b[k - 1] * (u[up] - u[dn]) - comp;
    const T t = sum + y;
    comp = (t - sum) - y;
    sum = t;
  }
#pragma unroll
  for (int off = 1; off < L; off <<= 1) {
    sum += __shfl_xor(sum, off);
    comp += __shfl_xor(comp, off);
  }
  return sum - comp;
}

// Lanes per grid point of the streaming kernels: the Fourier derivative's
// long sum is split over 8 lanes, the finite differences use one.
template <int ORDER>
struct PointLanes {
  static constexpr int L = ORDER == GBS_FD_SPECTRAL ? 8 : 1;
};

// Mode bits of one sequence in one leap-frog launch.
enum : int32_t {
  MODE_LAST = 1,    // s == N_j: average, combine, no level written
  MODE_FIRST = 2,   // first sequence to finish: acc = c y*
  MODE_FINAL = 4,   // last sequence to finish: y_out = acc + c y*
};

template <typename T>
struct SeqDesc {
  const T* cur;    // y_s
  const T* old;    // y_{s-1}
  T* out;          // y_{s+1} (overwrites old's buffer), unused when MODE_LAST
  T h2;            // 2 h_j
  int32_t mode;
  double cw;       // c_j
  double amp;      // source wavelet at t_0 + s h_j
};

struct SrcDesc {
  int64_t idx;     // within one field
  double w;
  int32_t rhs;
  int32_t pad;
};

// The point sources of right-hand side `rhs` in one lane's column, found
// once per wavefront: the blocked passes evaluate source terms only in
// wavefronts where some lane owns a source column (`any`, wave-uniform), and
// a lane with exactly one source compares rows against a register copy.
struct LaneSource {
  double w = 0.0;
  int row = -1;
  int count = 0;     // sources in this lane's column
  bool any = false;
};

__device__ __forceinline__ LaneSource lane_source(const SrcDesc* src, int nsrc, int64_t rhs, int gx,
                                                  int nx) {
  LaneSource ls;
  for (int k = 0; k < nsrc; ++k) {
    if (src[k].rhs == rhs && (int)(src[k].idx % nx) == gx) {
      ++ls.count;
      ls.row = (int)(src[k].idx / nx);
      ls.w = src[k].w;
    }
  }
  ls.any = __ballot(ls.count > 0) != 0;
  return ls;
}

struct Geometry {
  int32_t nx, ny, nz;
  int32_t nsrc;
  int64_t field;   // points per field
  int64_t state;   // elements per right-hand side (F * field)
  const void* fourier;   // Fourier-derivative weights b_k in the state's type, or null
};

template <typename T>
struct StepArgs {
  SeqDesc<T> seq[GBS_MAX_SEQ];
  SrcDesc src[GBS_MAX_SRC];
  Geometry g;
  double* acc;     // FP64 accumulator, state-sized
  T* yout;
  const T* c2f;    // coefficient field or null
  T c2c;           // constant coefficient
  T invx, invy, invz;
  int32_t tz;      // LDS-tiled 3-D sweeps: planes per block (0: the kernel's TZ)
};

template <typename T>
struct FirstArgs {
  T* out[GBS_MAX_SEQ];   // y_1 of every sequence
  T h[GBS_MAX_SEQ];
  SrcDesc src[GBS_MAX_SRC];
  Geometry g;
  const T* y0;
  const T* c2f;
  T c2c;
  T invx, invy, invz;
  int32_t nseq;
  int32_t tz;            // LDS-tiled 3-D sweeps: planes per block (0: the kernel's TZ)
  double amp;            // source wavelet at t_0
};

}  // namespace gbs
