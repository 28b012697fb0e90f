// Temporally blocked adjoint of one extrapolated GBS macro step, 2-D
// acoustic operator (FD4).
//
// The transpose of sequence j (leap-frog run backwards, see adjoint.hpp)
// needs the forward levels y_N .. y_1 in reverse order.  They are not
// stored: the forward recurrence y_{n+1} = y_{n-1} + 2h f(t_n, y_n) is
// reversible, y_{n-1} = y_{n+1} - 2h f(t_n, y_n), so the backward pass
// regenerates them from the pair (y_{N-1}, y_N) that a forward pass leaves
// (to rounding: the regenerated levels enter only the c^2 gradient).
//
// The adjoint is carried in the variables Psi = (c^2 lambda_p, lambda_v).
// With (A^T lambda)_p = div lambda_v and (A^T lambda)_v = grad(c^2 lambda_p),
// the transposed operator acting on Psi is
//   M Psi = (c^2 div lambda_v, grad Pi),   Pi = c^2 lambda_p,
// which is the acoustic operator with its sign flipped: the adjoint
// recurrence becomes a leap-frog on Psi with the same stencils as the
// forward one, and c^2 enters pointwise only.
//
// Levels: Z_k = (Y_k, Psi_k) with Y_k = y_{N-1-k} and Psi_k = Psi(lambda_{N-k})
// for k >= 0, and Z_{-1} = (y_N, U), U = Psi(c_j ybar / 2).  Then
//   Psi_0 = U + h M U          (the averaging's transpose, one Euler-like step)
//   Z_{k+1} = Z_{k-1} + 2h (-(A Y_k + s(t_{N-1-k})), M Psi_k),
// and the c^2 gradient of the sequence is
//   h lambda_{-1,p} (-div v(y_N)) + sum_{k=0}^{N-2} 2h lambda_{k,p} (-div v(Y_k)),
// summed per row as Pi times the divergence and divided by the row's c^2
// once.
// The last level gives lambda_1 (Z_{N-1}) and lambda_0 = lambda_2 (Z_{N-2}):
// the pass stores lambda_0 + lambda_1 and h lambda_1 in FP64, per sequence.
//
// Work layout as in the forward passes (temporal.hpp): one wavefront per
// 64-column strip and band, level e produced R rows behind level e-1, the
// 2R+1 rows of each level's six fields in registers, x-neighbours by
// cross-lane moves, halo columns recomputed.  The gradient of a row
// collects one term per level at different row steps: a small FP64 ring in
// LDS (one slot per row in flight) sums them, and the row's total is added
// to the sequence's gradient buffer once, when the last level has passed it.
#pragma once

#include "temporal.hpp"

namespace gbs {

constexpr int ADJ_FIRST = 1;   // input: ybar, y_N, y_{N-1}; evaluation 1 is the Euler-like step
constexpr int ADJ_FINAL = 2;   // output: lambda_0 + lambda_1 and h lambda_1 (FP64)

template <typename T>
struct AdjPassSeq {
  const T* cur;        // later pass: Z_s (Y then Psi, two states); first: y_N
  const T* old;        // later pass: Z_{s-1}; first: y_{N-1}
  const T* ybar;       // first pass: the adjoint at the macro step's end
  T* out_a;            // non-final: Z of level g-1
  T* out_b;            // non-final: Z of level g
  double* ysum;        // final: lambda_0 + lambda_1 (FP64 state)
  double* f1;          // final: h lambda_1 (FP64 state)
  double* gsum;        // the sequence's c^2 gradient, one FP64 field per right-hand side
  T h;                 // substep h_j
  T half_cw;           // c_j / 2
  int32_t g, flags, strips, pad;
  double amp[PASS_GMAX];   // source wavelet at each evaluation's time
};

template <typename T>
struct AdjPassArgs {
  AdjPassSeq<T> seq[GBS_MAX_SEQ];
  const SrcDesc* src_dev;
  Geometry g;
  const T* c2f;
  T c2c;
  T invx, invy;
  int64_t zstride;     // elements of one whole state (every right-hand side): Y to Psi
  int32_t band, nbands, max_strips;
};

template <typename T, int G, bool VARC>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2)))
void adj_pass2d(const AdjPassArgs<T> a) {
  constexpr int ORDER = 4;
  constexpr int R = Fd<ORDER>::R;
  constexpr int S = R;                               // rows between consecutive levels
  constexpr int P = 2 * R + 1;                       // window rows per level
  constexpr int CQ = G * S + 1;                      // rows in flight (c^2 and gradient rings)
  const AdjPassSeq<T>& d = a.seq[blockIdx.y];
  const int wq = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
  const int unit = __builtin_amdgcn_readfirstlane((int)(blockIdx.x * 4 + wq));
  const int strip = unit % a.max_strips;
  const int band = unit / a.max_strips;
  if (strip >= d.strips || band >= a.nbands) return;
  const int lane = threadIdx.x & 63;
  const int nx = a.g.nx, ny = a.g.ny;
  const int g = d.g;
  const int halo = g * R;
  const int x0 = strip * (64 - 2 * halo);
  const int col = x0 - halo + lane;
  const int gx = pmod(col, nx);
  const bool lane_ok = lane >= halo && lane < 64 - halo && col < nx;
  const int ya = band * a.band;
  const int yb = min(ya + a.band, ny);
  const int i0 = ya - halo;
  const int niter = (yb - ya) + halo + g * S;
  const int64_t base = (int64_t)blockIdx.z * a.g.state;
  const int64_t F1 = a.g.field, F2 = 2 * a.g.field, ST = a.zstride;
  const bool first = d.flags & ADJ_FIRST;
  const bool final_ = d.flags & ADJ_FINAL;
  const LaneSource ls =
      a.g.nsrc > 0 ? lane_source(a.src_dev, a.g.nsrc, blockIdx.z, gx, nx) : LaneSource();
  const bool srcs = ls.any;
  const T h = d.h, h2 = T(2) * d.h;
  const T invx = a.invx, invy = a.invy;
  // first pass: cur = y_N (Y of level 0), old = y_{N-1} (Y of level 1),
  // ybar gives Psi of level 0; later passes: cur / old hold Z (Y at +0,
  // Psi at +ST, ST = one whole state of every right-hand side)
  const T* __restrict__ cur = d.cur + base + gx;
  const T* __restrict__ old = d.old + base + gx;
  const T* __restrict__ yb_in = first ? d.ybar + base + gx : nullptr;
  const T* __restrict__ cpsi = first ? nullptr : cur + ST;
  const T* __restrict__ opsi = first ? nullptr : old + ST;

  __shared__ T c2q[VARC ? 4 : 1][VARC ? CQ : 1][64];
  __shared__ double gq[4][CQ][64];
  T* const myq = &c2q[VARC ? wq : 0][0][lane];
  double* const myg = &gq[wq][0][lane];
  if constexpr (VARC) {
    for (int s = 1; s < CQ; ++s) myq[(CQ - s) * 64] = a.c2f[(int64_t)pmod(i0 - s, ny) * nx + gx];
  }
  for (int s = 0; s < CQ; ++s) myg[s * 64] = 0.0;
  int kq = 0;

  T W[G][P][6];
#pragma unroll
  for (int e = 0; e < G; ++e)
#pragma unroll
    for (int s = 0; s < P; ++s)
#pragma unroll
      for (int q = 0; q < 6; ++q) W[e][s][q] = T(0);

  int irow = pmod(i0, ny);
  for (int kb = 0; kb < niter; kb += P) {
#pragma unroll
    for (int u = 0; u < P; ++u) {
      const int k = kb + u;
      // inputs: level 0 at row i; level -1 (later passes) or level 1's Y
      // (first pass) at the row level 1 updates now, i - S
      T om[6];
      // this row's c^2: in FP32 queued at the end of the row step (its first
      // reader is level 1, S row steps later), so that only a first pass,
      // which scales the injected adjoint by it, waits for the load here; in
      // FP64 holding it that long would spill (the kernel is at 256 VGPRs)
      T c2n = a.c2c;
      {
        const int64_t e0 = (int64_t)irow * nx;
        const int64_t e1 = (int64_t)wrap_sub(irow, S, ny) * nx;
        if constexpr (VARC) {
          c2n = a.c2f[e0 + gx];
          if constexpr (sizeof(T) == 8) myq[kq * 64] = c2n;
        }
        W[0][u][0] = cur[e0];
        W[0][u][1] = cur[e0 + F1];
        W[0][u][2] = cur[e0 + F2];
        if (first) {
          const T b0 = yb_in[e0], b1 = yb_in[e0 + F1], b2 = yb_in[e0 + F2];
          W[0][u][3] = c2n * (d.half_cw * b0);
          W[0][u][4] = d.half_cw * b1;
          W[0][u][5] = d.half_cw * b2;
          om[0] = old[e1];
          om[1] = old[e1 + F1];
          om[2] = old[e1 + F2];
          om[3] = om[4] = om[5] = T(0);
        } else {
          W[0][u][3] = cpsi[e0];
          W[0][u][4] = cpsi[e0 + F1];
          W[0][u][5] = cpsi[e0 + F2];
#pragma unroll
          for (int q = 0; q < 3; ++q) {
            om[q] = old[e1 + q * F1];
            om[3 + q] = opsi[e1 + q * F1];
          }
        }
      }
#pragma unroll
      for (int e = 1; e <= G; ++e) {
        if (e > g) continue;
        const int c = ((u - e * S) % P + P) % P;     // slot of row i - e S
        const T(&In)[P][6] = W[e - 1];
        T sy[4];                                     // y-sums of Y_p, Y_vy, Pi, lambda_y
        {
          const int up = (c + 1) % P, dn = (c - 1 + P) % P;
          sy[0] = Fd<ORDER>::template w<T>(0) * (In[up][0] - In[dn][0]);
          sy[1] = Fd<ORDER>::template w<T>(0) * (In[up][2] - In[dn][2]);
          sy[2] = Fd<ORDER>::template w<T>(0) * (In[up][3] - In[dn][3]);
          sy[3] = Fd<ORDER>::template w<T>(0) * (In[up][5] - In[dn][5]);
        }
#pragma unroll
        for (int kk = 1; kk < R; ++kk) {
          const int up = (c + kk + 1) % P, dn = (c - kk - 1 + 2 * P) % P;
          sy[0] += Fd<ORDER>::template w<T>(kk) * (In[up][0] - In[dn][0]);
          sy[1] += Fd<ORDER>::template w<T>(kk) * (In[up][2] - In[dn][2]);
          sy[2] += Fd<ORDER>::template w<T>(kk) * (In[up][3] - In[dn][3]);
          sy[3] += Fd<ORDER>::template w<T>(kk) * (In[up][5] - In[dn][5]);
        }
        const T sxp = lane_dsum<T, ORDER>(In[c][0]);
        const T sxv = lane_dsum<T, ORDER>(In[c][1]);
        const T sxP = lane_dsum<T, ORDER>(In[c][3]);
        const T sxL = lane_dsum<T, ORDER>(In[c][4]);
        int sl = kq - e * S;
        if (sl < 0) sl += CQ;
        T c2 = a.c2c;
        if constexpr (VARC) c2 = myq[sl * 64];
        // the row of this level's point, formed only where a source term or
        // the pass's stores need it
        auto level_row = [&]() { return wrap_sub(irow, e * S, ny); };
        // forward operator on Y (for the reversal), M on Psi
        const T dvx = invx * sxv;
        const T dvy = invy * sy[1];
        T fy[3], fm[3];
        fy[0] = -(c2 * (dvx + dvy));
        fy[1] = -(invx * sxp);
        fy[2] = -(invy * sy[0]);
        if (srcs) {
          const int row = level_row();
          if (ls.count == 1) {
            if (row == ls.row) fy[0] += (T)(ls.w * d.amp[e - 1]);
          } else if (ls.count > 1) {
            fy[0] += source_term<T>(a.src_dev, a.g.nsrc, blockIdx.z, (int64_t)row * nx + gx,
                                    d.amp[e - 1]);
          }
        }
        fm[0] = c2 * (invx * sxL + invy * sy[3]);
        fm[1] = invx * sxP;
        fm[2] = invy * sy[2];
        // c^2 gradient term of level e-1 (h for Z_{-1}, else 2h), times c^2:
        // lambda_p = Pi / c^2 is divided out once per row, at the flush
        {
          const double fac = (first && e == 1) ? (double)h : 2.0 * (double)h;
          myg[sl * 64] += fac * (double)In[c][3] * (-((double)dvx + (double)dvy));
        }
        T nw[6];
        if (e == 1 && first) {
#pragma unroll
          for (int q = 0; q < 3; ++q) {
            nw[q] = om[q];                                  // Y_0 = y_{N-1}
            nw[3 + q] = In[c][3 + q] + h * fm[q];           // Psi_0 = U + h M U
          }
        } else {
          const T* o = e == 1 ? om : W[e >= 2 ? e - 2 : 0][c];
#pragma unroll
          for (int q = 0; q < 3; ++q) {
            nw[q] = o[q] - h2 * fy[q];
            nw[3 + q] = o[3 + q] + h2 * fm[q];
          }
        }
        if (e == g) {
          const int yo = i0 + k - e * S;
          const int64_t pt = (int64_t)level_row() * nx + gx;
          const bool store = lane_ok && yo >= ya && yo < yb;
          if (store) {
            // the gradient row sum is read before the level stores: the
            // compiler cannot move the load across stores it may alias, and
            // behind them its wait would also wait for every store
            double* gp = d.gsum + (int64_t)blockIdx.z * F1 + pt;
            const double gold = first ? 0.0 : *gp;
            if (!final_) {
#pragma unroll
              for (int q = 0; q < 3; ++q) {
                // read back only by the next round's launch
                __builtin_nontemporal_store(In[c][q], d.out_a + base + pt + q * F1);
                __builtin_nontemporal_store(In[c][3 + q], d.out_a + base + ST + pt + q * F1);
                __builtin_nontemporal_store(nw[q], d.out_b + base + pt + q * F1);
                __builtin_nontemporal_store(nw[3 + q], d.out_b + base + ST + pt + q * F1);
              }
            } else {
              // lambda_1 = level g (Z_{N-1}), lambda_0 = level g-1 (Z_{N-2})
              const double l1[3] = {(double)nw[3] / (double)c2, (double)nw[4], (double)nw[5]};
              const double l0[3] = {(double)In[c][3] / (double)c2, (double)In[c][4],
                                    (double)In[c][5]};
#pragma unroll
              for (int q = 0; q < 3; ++q) {
                d.ysum[base + pt + q * F1] = l0[q] + l1[q];
                d.f1[base + pt + q * F1] = (double)h * l1[q];
              }
            }
            const double add = myg[sl * 64] / (double)c2;
            *gp = first ? add : gold + add;
          }
          myg[sl * 64] = 0.0;
        } else if (e < G) {
#pragma unroll
          for (int q = 0; q < 6; ++q) W[e][c][q] = nw[q];
        }
      }
      if constexpr (VARC && sizeof(T) == 4) myq[kq * 64] = c2n;
      irow = irow + 1 == ny ? 0 : irow + 1;
      kq = kq + 1 == CQ ? 0 : kq + 1;
    }
  }
}

}  // namespace gbs
