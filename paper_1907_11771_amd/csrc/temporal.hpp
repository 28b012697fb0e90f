// Temporally blocked GBS sequence passes for the 2-D acoustic operator.
//
// A pass advances one sequence by up to G evaluations of f in one launch, so
// that the intermediate levels never leave the chip.  The first pass of a
// sequence starts from y_0.  In the shared form (PASS_F0) the evaluation
// f(t_0, y_0) is done once per macro step by f0_march2d, as Sect. 3.6 shares
// it, and the first pass of every sequence starts from the pair
// (y_0, y_1 = y_0 + h F_0), formed as it loads its input rows; otherwise
// (PASS_FIRST) the first pass evaluates f(t_0, y_0) itself and performs the
// forward Euler step (Sect. 2.1, eq. GBS).  Later passes start from the two
// levels the previous pass stored.  The last pass applies the averaging
// y* = (y_{N-1} + 2 y_N + y_{N+1}) / 4 and stores y* in FP64; a separate
// kernel forms sum_j c_j y*_j in ascending N (Sect. 3.2), or, when the
// sequence with the largest N is the only one left in the last launch, its
// final pass does (PASS_COMBINE, kernels instantiated with COMB): at every
// output row it reads the other sequences' y* and stores y_out.
//
// Work layout: one wavefront owns a strip of 64 consecutive columns and a
// band of rows, and marches down the band.  Level A_e (e = 0 is the pass's
// input level) is produced e*R rows behind the input front (time skew), so
// that every stencil input of A_e already exists.  Each lane keeps, for
// every level, the last 2R+1 rows of (p, v_x, v_y) of its column in
// registers (y-neighbours); x-neighbours come from the adjacent lanes, by
// cross-lane moves, and in FP64 p's through a row in LDS that the wavefront
// writes and reads back.  The lanes next to the strip edges receive no valid
// neighbour data, so A_e is exact only on lanes [e*R, 64 - e*R): a pass of
// g evaluations stores the 64 - 2 g R inner columns, and consecutive strips
// overlap by 2 g R columns.
#pragma once

#include "stencil.hpp"

namespace gbs {

constexpr int PASS_FIRST = 1;   // input is y_0; evaluation 1 is forward Euler
constexpr int PASS_FINAL = 2;   // output is y* (FP64) instead of two levels
constexpr int PASS_KEEP = 4;    // final pass also stores (y_{N-1}, y_N) to out_a, out_b
                                // (only in kernels instantiated with KEEP = true)
constexpr int PASS_F0 = 8;      // first pass of the shared form: old = y_0, cur = y_0 + h F_0
constexpr int PASS_COMBINE = 16;  // final pass stores y_out = sum_j c_j y*_j (COMB kernels)
constexpr int PASS_GMAX = 8;
// the x-derivative of p from an LDS row of the wavefront instead of lane
// moves (WPG = 1 passes, FP64, where a lane move of one value takes two
// 32-bit moves)
template <typename T>
constexpr bool pass_xlds() { return sizeof(T) == 8; }
constexpr int COMB_MAX = 5;     // y* of other sequences a combining pass reads per point

template <typename T>
struct PassSeq {
  const T* old;       // later pass: y_{s-1}
  const T* cur;       // later pass: y_s; first pass: y_0
  T* out_a;           // non-final: A_{g-1}; final with PASS_KEEP: y_{N-1}
  T* out_b;           // non-final: A_g; final with PASS_KEEP: y_N
  double* ystar;      // final: y* (FP64, state-sized)
  T h;                // substep h_j
  int32_t g;          // evaluations in this pass (1..G)
  int32_t flags;
  int32_t strips;     // strips along x for this g
  int32_t hs;         // recomputed columns on each side of a strip, >= g R (0: g R)
  double amp[PASS_GMAX];  // source wavelet at each evaluation's time
};

// The combination a PASS_COMBINE pass forms: y_out = sum_r c[r] y*_r (the
// other sequences, ascending N) + c_last y*_this, summed in that order.
template <typename T>
struct CombineTail {
  const double* ystar[COMB_MAX];
  double c[COMB_MAX];
  double c_last;
  T* yout;
  int32_t n;          // sequences in ystar (1..COMB_MAX)
};

template <typename T>
struct PassArgs {
  PassSeq<T> seq[GBS_MAX_SEQ];
  const SrcDesc* src_dev;    // device copy of the point sources
  Geometry g;
  const T* c2f;
  const T* f0;        // F_0 = f(t_0, y_0) for PASS_F0 passes (state-sized) or null
  T c2c;
  T invx, invy;
  int32_t band;       // rows per band
  int32_t nbands;
  int32_t max_strips;
  // order of the workgroups (WPG = 1): 0: blockIdx.y is the sequence;
  // 1, 2: a 1-D grid in which the nseq sequences of one group of 4 units
  // (4 strips of a band) are consecutive workgroups of one XCD (workgroups
  // go to the 8 XCDs round-robin), so that first passes reading the same
  // y_0 rows share that XCD's L2; groups round-robin over the XCDs (1) or
  // contiguous per XCD, `per` groups each (2)
  int32_t order, nseq, per;
  CombineTail<T> comb;
};

// Cross-lane moves over the whole wavefront: lane l receives the value of
// lane l+1 (from_right) or l-1 (from_left); the edge lane receives 0, which
// only ever feeds the discarded halo lanes.
template <int CTRL>
__device__ __forceinline__ float lane_move(float v) {
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, 0xF, 0xF, true));
}
template <int CTRL>
__device__ __forceinline__ double lane_move(double v) {
  return __longlong_as_double(
      __builtin_amdgcn_update_dpp(0ll, __double_as_longlong(v), CTRL, 0xF, 0xF, true));
}
constexpr int DPP_WAVE_SHL1 = 0x130;   // lane l <- lane l+1
constexpr int DPP_WAVE_SHR1 = 0x138;   // lane l <- lane l-1

// sum_k W_k (u(x+k) - u(x-k)) with u(x +/- k) gathered from the lanes
// at distance k.
template <typename T, int ORDER>
__device__ __forceinline__ T lane_dsum(T u) {
  constexpr int R = Fd<ORDER>::R;
  T up = lane_move<DPP_WAVE_SHL1>(u), dn = lane_move<DPP_WAVE_SHR1>(u);
  T s = Fd<ORDER>::template w<T>(0) * (up - dn);
#pragma unroll
  for (int k = 1; k < R; ++k) {
    up = lane_move<DPP_WAVE_SHL1>(up);
    dn = lane_move<DPP_WAVE_SHR1>(dn);
    s += Fd<ORDER>::template w<T>(k) * (up - dn);
  }
  return s;
}

// r - d wrapped into [0, n) for 0 <= r < n, d >= 0 (wave-uniform operands);
// one addition when d <= n, the common case
__device__ __forceinline__ int wrap_sub(int r, int d, int n) {
  r -= d;
  if (r < 0) {
    r += n;
    while (r < 0) r += n;
  }
  return r;
}

// Everything one wavefront needs for its part of a pass, by value.
template <typename T>
struct PassWork {
  const T* cur;        // later pass: y_s; first pass: y_0   (this right-hand side)
  const T* old;        // later pass: y_{s-1}
  T* out_a;            // non-final: A_{g-1}
  T* out_b;            // non-final: A_g
  double* ystar;       // final: y* (FP64)
  const T* c2f;        // coefficient field or null
  const T* f0;         // PASS_F0: F_0 of this right-hand side
  const CombineTail<T>* comb;   // PASS_COMBINE: the combination (kernel arguments)
  int64_t rhs_off;     // PASS_COMBINE: offset of this right-hand side's state
  const SrcDesc* src;  // device array of point sources (global memory) or null
  int64_t field;       // points per field
  int64_t rhs;         // right-hand-side index (for sources)
  T h, c2c, invx, invy;
  int32_t nx, ny, g, flags, band, nsrc;
  int32_t hs;          // strip halo in columns, >= g R (0: g R)
  double amp[PASS_GMAX];
};

// A workgroup's pass over its strip and band.
//
// The workgroup's WPG wavefronts cover 64 * WPG consecutive columns; wave v
// holds columns x0 - g R + 64 v + lane.  Inside a wavefront x-neighbours come
// from adjacent lanes (DPP wave shifts); across wavefront boundaries the R
// edge lanes of every level row are exchanged through a small LDS ring (the
// value a level needs from its neighbour was produced S row steps earlier,
// so one barrier per row step suffices).  Only the workgroup's outer g R
// columns on each side are recomputed halo.
//
// Time skew between consecutive levels: with SKEW1 = false level e is
// produced R rows behind level e-1 and the levels of one row step are
// evaluated in ascending order (each uses the row its predecessor has just
// produced); with SKEW1 = true the skew is R+1 rows and the levels are
// evaluated in descending order, so that all of them read only rows
// produced in earlier row steps (independent work within a row step), at the
// cost of one more window row per level.  The number of evaluations g of a
// pass (at most G) is a runtime value, uniform over the workgroup.
template <typename T, int R, int G, int S, int WPG>
struct EdgeRing {
  // [slot][wave][level][field p/vx][R left lanes, R right lanes]
  T v[S + 1][WPG][G][2][2 * R];
};

// x-derivative sum with the lanes beyond this wavefront's edges supplied
// by its neighbours' edge values (left: lanes 64-R..63, right: lanes 0..R-1).
template <typename T, int ORDER>
__device__ __forceinline__ T lane_dsum_edges(T u, int lane, const T* left, const T* right,
                                             bool has_left, bool has_right) {
  constexpr int R = Fd<ORDER>::R;
  T up = lane_move<DPP_WAVE_SHL1>(u), dn = lane_move<DPP_WAVE_SHR1>(u);
  if (has_right && lane == 63) up = right[0];
  if (has_left && lane == 0) dn = left[R - 1];
  T s = Fd<ORDER>::template w<T>(0) * (up - dn);
#pragma unroll
  for (int k = 1; k < R; ++k) {
    up = lane_move<DPP_WAVE_SHL1>(up);
    dn = lane_move<DPP_WAVE_SHR1>(dn);
    if (has_right && lane == 63) up = right[k];
    if (has_left && lane == 0) dn = left[R - 1 - k];
    s += Fd<ORDER>::template w<T>(k) * (up - dn);
  }
  return s;
}

template <typename T, int ORDER, int G, bool SKEW1, int WPG, bool VARC, bool KEEP = false,
          bool COMB = false>
__device__ __forceinline__ void pass_body(const PassWork<T> w, const int strip, const int band) {
  constexpr int R = Fd<ORDER>::R;
  constexpr int S = SKEW1 ? R + 1 : R;               // rows between consecutive levels
  constexpr int P = SKEW1 ? 2 * R + 2 : 2 * R + 1;   // window rows per level
  __shared__ EdgeRing<T, R, G, S, WPG> ring;
  const int lane = threadIdx.x & 63;
  const int wave = WPG > 1 ? __builtin_amdgcn_readfirstlane(threadIdx.x >> 6) : 0;
  const int nx = w.nx, ny = w.ny;
  const int g = w.g;
  const int halo = g * R;                            // rows the levels trail (y)
  // recomputed columns on each side of the strip: g R, or more where the
  // passes of one launch share one strip geometry (A_g is exact on lanes
  // [g R, 64 - g R), so any wider halo stores exact values)
  const int hxs = w.hs > halo ? w.hs : halo;
  const int wv = 64 * WPG - 2 * hxs;
  const int x0 = strip * wv;
  const int col = x0 - hxs + 64 * wave + lane;       // unwrapped column of this lane
  const int gx = pmod(col, nx);
  const int gl = 64 * wave + lane;                   // lane within the workgroup
  const bool lane_ok = gl >= hxs && gl < 64 * WPG - hxs && col < nx;
  const bool has_left = WPG > 1 && wave > 0, has_right = WPG > 1 && wave < WPG - 1;
  const bool edge_lane = lane < R || lane >= 64 - R;
  const int edge_idx = lane < R ? lane : R + lane - (64 - R);
  const int ya = band * w.band;
  const int yb = min(ya + w.band, ny);
  const int i0 = ya - halo;                          // first input row (A_0)
  const int niter = (yb - ya) + halo + g * S;        // until A_g reaches row yb - 1
  const int64_t F1 = w.field, F2 = 2 * w.field;
  const bool first = w.flags & PASS_FIRST;
  const bool f0mode = w.flags & PASS_F0;             // old = y_0, cur = y_0 + h F_0
  const bool final_ = w.flags & PASS_FINAL;
  const bool keep = KEEP && (w.flags & PASS_KEEP);   // compiled only where asked for
  const bool comb = COMB && (w.flags & PASS_COMBINE);
  constexpr bool varc = VARC;                       // c^2 field (else the constant)
  const LaneSource ls = w.nsrc > 0 ? lane_source(w.src, w.nsrc, w.rhs, gx, nx) : LaneSource();
  const bool srcs = ls.any;
  const T fac_lf = T(2) * w.h;
  const T* __restrict__ cur = w.cur + gx;
  const T* __restrict__ old = (first || f0mode) ? cur : w.old + gx;
  const T* __restrict__ f0p = f0mode ? w.f0 + gx : nullptr;
  // PASS_COMBINE: the other sequences' y* at the next output row, loaded one
  // row step before they are summed
  double pre[COMB ? COMB_MAX : 1][3];
  const int ncomb = comb ? w.comb->n : 0;
  auto prefetch = [&](int yr) {
    if constexpr (COMB) {
      const int64_t pn = w.rhs_off + (int64_t)yr * nx + gx;
#pragma unroll
      for (int r = 0; r < COMB_MAX; ++r)
        if (r < ncomb) {
          const double* yp = w.comb->ystar[r] + pn;
#pragma unroll
          for (int q = 0; q < 3; ++q) pre[r][q] = __builtin_nontemporal_load(yp + q * F1);
        }
    }
  };

  T W[G][P][3];
#pragma unroll
  for (int e = 0; e < G; ++e)
#pragma unroll
    for (int s = 0; s < P; ++s)
#pragma unroll
      for (int q = 0; q < 3; ++q) W[e][s][q] = T(0);

  // c^2 queue in LDS, one per wavefront: the coefficient row is loaded once,
  // with the input row, and level e reads it e S row steps later (a slot per
  // lane, so no barrier).  Pre-filled with the rows above the first input row.
  constexpr int CQ = G * S + 1;
  constexpr int NWQ = WPG > 1 ? WPG : 4;
  __shared__ T c2q[VARC ? NWQ : 1][VARC ? CQ : 1][64];
  const int wq = WPG > 1 ? wave : __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
  T* const myq = &c2q[VARC ? wq : 0][0][lane];
  // one row of p per wavefront for the x-neighbours (pass_xlds), R entries
  // of padding on each side feed only the discarded edge lanes
  constexpr bool XL = pass_xlds<T>() && WPG == 1;
  __shared__ T xrows[XL ? 4 : 1][XL ? 64 + 2 * R : 1];
  T* const xrow = &xrows[XL ? wq : 0][XL ? R : 0];
  if constexpr (VARC) {
    for (int s = 1; s < CQ; ++s) myq[(CQ - s) * 64] = w.c2f[(int64_t)pmod(i0 - s, ny) * nx + gx];
  }
  int kq = 0;                                        // row step modulo CQ

  int irow = pmod(i0, ny);                           // wrapped row of A_0 at this row step
  for (int kb = 0; kb < niter; kb += P) {
#pragma unroll
    for (int u = 0; u < P; ++u) {
      const int k = kb + u;                          // row step; A_0 row i = i0 + k
      // ring slots: written now, and produced S steps ago (read now)
      const int wslot = k % (S + 1), rslot = (k + 1) % (S + 1);
      // input rows: A_0 at row i, and for a later pass A_{-1} at the row
      // level 1 updates in this step
      T nxt[3], om[3];
      T c2new = T(0);   // this row's c^2, queued at the end of the row step (its first
                        // reader is level 1, S row steps later), so that its load
                        // does not stall the levels evaluated now
      {
        const int64_t e0 = (int64_t)irow * nx;
        nxt[0] = cur[e0];
        nxt[1] = cur[e0 + F1];
        nxt[2] = cur[e0 + F2];
        if (f0mode) {
          // y_1 = y_0 + h F_0, the forward Euler step every sequence shares
          // the evaluation of
          const T f0v[3] = {f0p[e0], f0p[e0 + F1], f0p[e0 + F2]};
#pragma unroll
          for (int q = 0; q < 3; ++q) nxt[q] = nxt[q] + w.h * f0v[q];
        }
        if constexpr (VARC) c2new = w.c2f[e0 + gx];
        if (!first) {
          const int64_t e1 = (int64_t)wrap_sub(irow, S, ny) * nx;
          om[0] = old[e1];
          om[1] = old[e1 + F1];
          om[2] = old[e1 + F2];
        } else {
          om[0] = om[1] = om[2] = T(0);
        }
      }
      if constexpr (WPG > 1) {
        if (edge_lane) {
          ring.v[wslot][wave][0][0][edge_idx] = nxt[0];
          ring.v[wslot][wave][0][1][edge_idx] = nxt[1];
        }
      }
      if constexpr (!SKEW1) {
#pragma unroll
        for (int q = 0; q < 3; ++q) W[0][u][q] = nxt[q];
      }
#pragma unroll
      for (int ee = 1; ee <= G; ++ee) {
        const int e = SKEW1 ? G + 1 - ee : ee;       // level evaluated now
        if (e > g) continue;
        const int c = ((u - e * S) % P + P) % P;     // slot of row i - e S
        const T(&In)[P][3] = W[e - 1];
        T syp, syv;
        {
          const int up = (c + 1) % P, dn = (c - 1 + P) % P;
          syp = Fd<ORDER>::template w<T>(0) * (In[up][0] - In[dn][0]);
          syv = Fd<ORDER>::template w<T>(0) * (In[up][2] - In[dn][2]);
        }
#pragma unroll
        for (int kk = 1; kk < R; ++kk) {
          const int up = (c + kk + 1) % P, dn = (c - kk - 1 + 2 * P) % P;
          syp += Fd<ORDER>::template w<T>(kk) * (In[up][0] - In[dn][0]);
          syv += Fd<ORDER>::template w<T>(kk) * (In[up][2] - In[dn][2]);
        }
        T sxp, sxv;
        if constexpr (WPG > 1) {
          // neighbours' edge values of level e-1's row i - e S (produced S
          // row steps ago)
          const int lw = has_left ? wave - 1 : wave, rw = has_right ? wave + 1 : wave;
          sxp = lane_dsum_edges<T, ORDER>(In[c][0], lane, &ring.v[rslot][lw][e - 1][0][R],
                                          &ring.v[rslot][rw][e - 1][0][0], has_left, has_right);
          sxv = lane_dsum_edges<T, ORDER>(In[c][1], lane, &ring.v[rslot][lw][e - 1][1][R],
                                          &ring.v[rslot][rw][e - 1][1][0], has_left, has_right);
        } else if constexpr (pass_xlds<T>()) {
          // p's x-neighbours through this wavefront's LDS row, v_x's by lane
          // moves: half the cross-lane traffic leaves the vector ALU.  The
          // row is written and read by one wavefront, whose LDS operations
          // execute in order, so no barrier; the wave barriers keep the
          // compiler from moving the other lanes' reads across the write (or
          // the next level's write across these reads), which a single
          // thread's view of the addresses would allow.
          xrow[lane] = In[c][0];
          __builtin_amdgcn_wave_barrier();
          T xn[2 * R];
#pragma unroll
          for (int kk = 0; kk < R; ++kk) {
            xn[2 * kk] = xrow[lane + kk + 1];
            xn[2 * kk + 1] = xrow[lane - kk - 1];
          }
          __builtin_amdgcn_wave_barrier();
          sxp = Fd<ORDER>::template w<T>(0) * (xn[0] - xn[1]);
#pragma unroll
          for (int kk = 1; kk < R; ++kk)
            sxp += Fd<ORDER>::template w<T>(kk) * (xn[2 * kk] - xn[2 * kk + 1]);
          sxv = lane_dsum<T, ORDER>(In[c][1]);
        } else {
          sxp = lane_dsum<T, ORDER>(In[c][0]);
          sxv = lane_dsum<T, ORDER>(In[c][1]);
        }
        // the row of this level's point and its flat index, formed only
        // where a source term or the pass's stores need them
        auto level_row = [&]() { return wrap_sub(irow, e * S, ny); };
        T c2 = w.c2c;
        if constexpr (VARC) {
          int sl = kq - e * S;
          if (sl < 0) sl += CQ;
          c2 = myq[sl * 64];
        }
        const T dvx = w.invx * sxv;
        const T dvy = w.invy * syv;
        T f[3];
        f[0] = -(c2 * (dvx + dvy));
        f[1] = -(w.invx * sxp);
        f[2] = -(w.invy * syp);
        if (srcs) {
          const int row = level_row();
          if (ls.count == 1) {
            if (row == ls.row) f[0] += (T)(ls.w * w.amp[e - 1]);
          } else if (ls.count > 1) {
            f[0] += source_term<T>(w.src, w.nsrc, w.rhs, (int64_t)row * nx + gx, w.amp[e - 1]);
          }
        }
        T nw[3];
        if (e == 1) {
          if (first) {
#pragma unroll
            for (int q = 0; q < 3; ++q) nw[q] = In[c][q] + w.h * f[q];        // forward Euler
          } else {
#pragma unroll
            for (int q = 0; q < 3; ++q) nw[q] = om[q] + fac_lf * f[q];         // leap-frog
          }
        } else {
#pragma unroll
          for (int q = 0; q < 3; ++q) nw[q] = W[e >= 2 ? e - 2 : 0][c][q] + fac_lf * f[q];
        }
        if (e == g) {
          // the pass's last level, at row i - g S
          const int yo = i0 + k - e * S;
          const int64_t pt = (int64_t)level_row() * nx + gx;
          if (lane_ok && yo >= ya && yo < yb) {
            if (!final_) {
#pragma unroll
              for (int q = 0; q < 3; ++q) {
                __builtin_nontemporal_store(In[c][q], w.out_a + pt + q * F1);
                __builtin_nontemporal_store(nw[q], w.out_b + pt + q * F1);
              }
            } else {
#pragma unroll
              for (int q = 0; q < 3; ++q) {
                const T ym1 = (e >= 2) ? W[e >= 2 ? e - 2 : 0][c][q] : (first ? In[c][q] : om[q]);
                const double ys = 0.25 * (((double)ym1 + 2.0 * (double)In[c][q]) + (double)nw[q]);
                if (comb) {
                  // y_out = sum_r c_r y*_r + c_last y*, in ascending N
                  double v = w.comb->c[0] * pre[0][q];
#pragma unroll
                  for (int r = 1; r < COMB_MAX; ++r)
                    if (r < ncomb) v = v + w.comb->c[r] * pre[r][q];
                  v = v + w.comb->c_last * ys;
                  w.comb->yout[w.rhs_off + pt + q * F1] = (T)v;
                } else {
                  __builtin_nontemporal_store(ys, w.ystar + pt + q * F1);
                }
                if (keep) {
                  w.out_a[pt + q * F1] = ym1;
                  w.out_b[pt + q * F1] = In[c][q];
                }
              }
            }
          }
          if (comb && lane_ok && yo + 1 >= ya && yo + 1 < yb) prefetch(yo + 1);
        } else if (e < G) {
#pragma unroll
          for (int q = 0; q < 3; ++q) W[e][c][q] = nw[q];
          if constexpr (WPG > 1) {
            if (edge_lane) {
              ring.v[wslot][wave][e][0][edge_idx] = nw[0];
              ring.v[wslot][wave][e][1][edge_idx] = nw[1];
            }
          }
        }
      }
      if constexpr (SKEW1) {
#pragma unroll
        for (int q = 0; q < 3; ++q) W[0][u][q] = nxt[q];
      }
      if constexpr (VARC) myq[kq * 64] = c2new;
      irow = irow + 1 == ny ? 0 : irow + 1;
      kq = kq + 1 == CQ ? 0 : kq + 1;
      if constexpr (WPG > 1) __syncthreads();
    }
  }
}

// One problem: blockIdx.y selects the sequence (its descriptor in the kernel
// arguments), blockIdx.z the right-hand side; a workgroup of WPG wavefronts
// covers one (strip, band), or with WPG = 1 each wavefront of a 4-wave block
// does.
template <typename T, int ORDER, int G, bool SKEW1, int WPG, bool VARC, bool KEEP = false,
          bool COMB = false>
__global__ __launch_bounds__(WPG > 1 ? 64 * WPG : 256) __attribute__((amdgpu_waves_per_eu(2)))
void pass2d(const PassArgs<T> a) {
  int seq = blockIdx.y, grp = blockIdx.x;
  if (WPG == 1 && a.order) {
    const int b = blockIdx.x, xcd = b & 7, k = b >> 3;
    seq = k % a.nseq;
    grp = a.order == 1 ? xcd + 8 * (k / a.nseq) : xcd * a.per + k / a.nseq;
  }
  const PassSeq<T>& d = a.seq[seq];
  const int unit = WPG > 1 ? (int)blockIdx.x
                           : __builtin_amdgcn_readfirstlane(grp * 4 + (threadIdx.x >> 6));
  const int strip = unit % a.max_strips;
  const int band = unit / a.max_strips;
  if (strip >= d.strips || band >= a.nbands) return;
  const int64_t base = (int64_t)blockIdx.z * a.g.state;
  PassWork<T> w;
  w.cur = d.cur + base;
  w.old = d.old ? d.old + base : nullptr;
  w.out_a = d.out_a + base;
  w.out_b = d.out_b + base;
  w.ystar = d.ystar ? d.ystar + base : nullptr;
  w.c2f = a.c2f;
  w.f0 = a.f0 ? a.f0 + base : nullptr;
  w.comb = &a.comb;
  w.rhs_off = base;
  w.src = a.src_dev;
  w.field = a.g.field;
  w.rhs = blockIdx.z;
  w.h = d.h;
  w.c2c = a.c2c;
  w.invx = a.invx;
  w.invy = a.invy;
  w.nx = a.g.nx;
  w.ny = a.g.ny;
  w.g = d.g;
  w.flags = d.flags;
  w.band = a.band;
  w.nsrc = a.g.nsrc;
  w.hs = WPG == 1 ? d.hs : 0;
#pragma unroll
  for (int e = 0; e < PASS_GMAX; ++e) w.amp[e] = d.amp[e];
  pass_body<T, ORDER, G, SKEW1, WPG, VARC, KEEP, COMB>(w, strip, band);
}

// F_0 = f(t_0, y_0) of the 2-D acoustic operator, with the sources at t_0:
// the one evaluation all sequences' forward Euler steps share (Sect. 3.6),
// written to a state-sized buffer for the first passes of the shared form.
// A 256-thread block covers 64 columns x 4 strips of TY rows; every thread
// walks down its column keeping the rows y-R..y+R of p and v_y in registers
// (the y-derivatives); the x-derivatives read the current row.  The same
// stencil sums, in the same order, as the passes' evaluations.
template <typename T>
struct F0Args {
  const T* y0;
  T* f0;
  const T* c2f;
  const SrcDesc* src;
  Geometry g;
  T c2c, invx, invy;
  double amp;          // source wavelet at t_0
};

template <typename T, int ORDER, int TY>
__global__ __launch_bounds__(256) void f0_march2d(const F0Args<T> a) {
  constexpr int R = Fd<ORDER>::R;
  const int nx = a.g.nx, ny = a.g.ny;
  const int ntx = (nx + 63) >> 6;
  const int tile = xcd_tile(blockIdx.x, gridDim.x);
  const int tx = tile % ntx, ty = tile / ntx;
  const int x = tx * 64 + (threadIdx.x & 63);
  const int y0 = ty * 4 * TY + (threadIdx.x >> 6) * TY;
  if (x >= nx || y0 >= ny) return;
  const int64_t rhs = blockIdx.z;
  const int64_t base = rhs * a.g.state;
  const int64_t F1 = a.g.field, F2 = 2 * a.g.field;
  const T* __restrict__ cp = a.y0 + base;
  const T* __restrict__ cvx = cp + F1;
  const T* __restrict__ cvy = cp + F2;
  T* __restrict__ out = a.f0 + base;
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
    T syp = Fd<ORDER>::template w<T>(0) * (pw[R + 1] - pw[R - 1]);
    T syv = Fd<ORDER>::template w<T>(0) * (vw[R + 1] - vw[R - 1]);
#pragma unroll
    for (int k = 1; k < R; ++k) {
      syp += Fd<ORDER>::template w<T>(k) * (pw[R + 1 + k] - pw[R - 1 - k]);
      syv += Fd<ORDER>::template w<T>(k) * (vw[R + 1 + k] - vw[R - 1 - k]);
    }
    const T sxp = dsum<T, ORDER>(cp + rowoff, x, nx, 1);
    const T sxv = dsum<T, ORDER>(cvx + rowoff, x, nx, 1);
    const T c2 = a.c2f ? a.c2f[rowoff + x] : a.c2c;
    const T dvx = a.invx * sxv;
    const T dvy = a.invy * syv;
    const int64_t idx = rowoff + x;
    T f0 = -(c2 * (dvx + dvy));
    if (a.g.nsrc) f0 += source_term<T>(a.src, a.g.nsrc, rhs, idx, a.amp);
    out[idx] = f0;
    out[idx + F1] = -(a.invx * sxp);
    out[idx + F2] = -(a.invy * syp);
#pragma unroll
    for (int k = 0; k < 2 * R; ++k) {
      pw[k] = pw[k + 1];
      vw[k] = vw[k + 1];
    }
  }
}

// A batch of problems: the passes of one round of every (instance, sequence)
// are items of a device table; unit u (a wavefront, or a workgroup of WPG
// wavefronts) belongs to the item whose first unit is the largest
// unit_begin <= u.
template <typename T>
struct PassItem {
  const T* cur;
  const T* old;
  T* out_a;
  T* out_b;
  double* ystar;
  const T* c2f;
  int64_t field;
  T h, c2c, invx, invy;
  int32_t nx, ny, g, flags, strips, nbands, band, wave_begin;
};

template <typename T>
struct BatchPassArgs {
  const PassItem<T>* items;
  int32_t n_items;
  int32_t total_waves;
};

template <typename T, int ORDER, int G, bool SKEW1, int WPG>
__global__ __launch_bounds__(WPG > 1 ? 64 * WPG : 256) __attribute__((amdgpu_waves_per_eu(2)))
void pass2d_batch(const BatchPassArgs<T> a) {
  const int unit = WPG > 1 ? (int)blockIdx.x
                           : __builtin_amdgcn_readfirstlane(blockIdx.x * 4 + (threadIdx.x >> 6));
  if (unit >= a.total_waves) return;
  int lo = 0, hi = a.n_items - 1;
  while (lo < hi) {                                  // last item with wave_begin <= unit
    const int mid = (lo + hi + 1) >> 1;
    if (a.items[mid].wave_begin <= unit) lo = mid; else hi = mid - 1;
  }
  const PassItem<T>* it = a.items + lo;
  const int local = unit - it->wave_begin;
  const int strips = it->strips;
  PassWork<T> w;
  w.cur = it->cur;
  w.old = it->old;
  w.out_a = it->out_a;
  w.out_b = it->out_b;
  w.ystar = it->ystar;
  w.c2f = it->c2f;
  w.f0 = nullptr;
  w.comb = nullptr;
  w.rhs_off = 0;
  w.src = nullptr;
  w.field = it->field;
  w.rhs = 0;
  w.h = it->h;
  w.c2c = it->c2c;
  w.invx = it->invx;
  w.invy = it->invy;
  w.nx = it->nx;
  w.ny = it->ny;
  w.g = it->g;
  w.flags = it->flags;
  w.band = it->band;
  w.nsrc = 0;
  w.hs = 0;
#pragma unroll
  for (int e = 0; e < PASS_GMAX; ++e) w.amp[e] = 0.0;
  if (w.c2f)
    pass_body<T, ORDER, G, SKEW1, WPG, true>(w, local % strips, local / strips);
  else
    pass_body<T, ORDER, G, SKEW1, WPG, false>(w, local % strips, local / strips);
}

// y_out = sum_j c_j y*_j, j in ascending N, accumulated in FP64.
template <typename T>
struct CombineArgs {
  const double* ystar[GBS_MAX_SEQ];
  double c[GBS_MAX_SEQ];
  T* yout;
  int64_t n;
  int32_t k;
};

// sum_j c[j] ystar[j][i] over j = 0..k-1 in ascending j.  The loads of up to
// COMBINE_CHUNK sequences are issued together before the sum uses them (a
// loop over the runtime k alone waits for each load before issuing the
// next); the sum itself keeps the order.  Each y* is read once: non-temporal
// loads keep them from displacing y_out, which the next macro step's first
// passes read.
constexpr int COMBINE_CHUNK = 8;

__device__ __forceinline__ double combine_point(const double* const* ystar, const double* c,
                                                int k, int64_t i) {
  double v = 0.0;
  for (int j0 = 0; j0 < k; j0 += COMBINE_CHUNK) {
    double y[COMBINE_CHUNK];
#pragma unroll
    for (int u = 0; u < COMBINE_CHUNK; ++u)
      y[u] = j0 + u < k ? __builtin_nontemporal_load(ystar[j0 + u] + i) : 0.0;
#pragma unroll
    for (int u = 0; u < COMBINE_CHUNK; ++u)
      if (j0 + u < k) v = j0 + u == 0 ? c[0] * y[u] : v + c[j0 + u] * y[u];
  }
  return v;
}

template <typename T>
__global__ __launch_bounds__(256) void combine_kernel(const CombineArgs<T> a) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= a.n) return;
  a.yout[i] = (T)combine_point(a.ystar, a.c, a.k, i);
}

// The same for a batch: block b belongs to the instance whose first block is
// the largest block_begin <= b.
template <typename T>
struct CombineItem {
  const double* ystar[GBS_MAX_SEQ];
  double c[GBS_MAX_SEQ];
  T* yout;
  int64_t n;
  int32_t k;
  int32_t block_begin;
};

template <typename T>
__global__ __launch_bounds__(256) void combine_batch(const CombineItem<T>* items, int n_items,
                                                     int total_blocks) {
  const int b = blockIdx.x;
  if (b >= total_blocks) return;
  int lo = 0, hi = n_items - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (items[mid].block_begin <= b) lo = mid; else hi = mid - 1;
  }
  const CombineItem<T>* it = items + lo;
  const int64_t i = (int64_t)(b - it->block_begin) * blockDim.x + threadIdx.x;
  if (i >= it->n) return;
  it->yout[i] = (T)combine_point(it->ystar, it->c, it->k, i);
}

}  // namespace gbs
