// Plan creation, validation and the macro-step launch schedule.
//
// Per macro step (Sect. 2.1 eq. GBS, Sect. 3.2, Sect. 3.6):
//   first_kernel  : F_0 = f(t_0, y_0) once, y_1 = y_0 + h_j F_0 for all j
//   lf_kernel(s)  : for s = 1..N_max, every sequence with N_j >= s advances
//                   one leap-frog step; at s = N_j it averages and adds
//                   c_j y*_j to the FP64 accumulator (the last one writes
//                   y_out).
// 1 + N_max launches and 1 + sum_j N_j evaluations of f per macro step.
//
// Workspace layout (caller-owned device memory, 256-byte aligned pieces):
//   acc            FP64, R * F * points
//   level[j][0..1] dtype, R * F * points each (two leap-frog levels; the new
//                  level overwrites the older one in place)
#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <new>
#include <string>
#include <tuple>
#include <vector>

#include "internal.hpp"
#include "kernels.hpp"
#include "temporal.hpp"
#include "adjoint.hpp"
#include "adjoint_blocked.hpp"

namespace gbs {

static thread_local std::string g_last_error;

int fail(int status, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  g_last_error = buf;
  return status;
}

}  // namespace gbs

using namespace gbs;

struct EventPair {
  hipEvent_t a = nullptr, b = nullptr;
};

constexpr int GBS_MAX_LANES = 4;

struct gbs_plan {
  gbs_problem prob;
  int k = 0;
  int32_t steps[GBS_MAX_SEQ];
  double w[GBS_MAX_SEQ];
  int order[GBS_MAX_SEQ];  // sequence indices by ascending N
  int nmax = 0;
  double H = 0;
  int F = 0;
  int64_t field = 0, state = 0;
  hipStream_t stream = nullptr;
  double* acc = nullptr;
  void* lev[GBS_MAX_SEQ][2];
  // sources (host copy, and a device copy at the start of the workspace)
  int nsrc = 0;
  SrcDesc src[GBS_MAX_SRC];
  SrcDesc* src_dev = nullptr;
  // receivers (device table in the workspace)
  int nrec = 0;
  bool rec_distinct = true;   // no two receivers share a (rhs, point)
  RecDesc* rec_dev = nullptr;
  double f0 = 0, delay = 0;
  // Fourier-derivative weights (spectral advection): host copy in the
  // state's type, device copy in the workspace, uploaded before the first step
  std::vector<unsigned char> fourier_host;
  void* fourier_dev = nullptr;
  bool fourier_ready = false;
  // leap-frog kernel variant (GBS_VARIANT_*) and rows per band of the
  // temporally blocked passes
  int variant = 0;
  int band = 0;            // 0: chosen per launch
  int wave_order = 0;      // workgroup order of the blocked passes (PassArgs::order)
  int form = 0;            // GBS_FORM_* flags of the blocked passes
  // temporally blocked layout: per sequence two pairs of levels
  void* pair[GBS_MAX_SEQ][2][2];
  // gbs_step_keep_pairs: caller's buffer for (y_{N-1}, y_N) of every
  // sequence and macro step, set for the duration of that call only
  void* keep_out = nullptr;
  // the blocked passes of one macro step spread over `lanes` streams (the
  // plan's stream and lanes - 1 streams of its own), joined before the
  // combination
  int lanes = 1;
  hipStream_t lane_stream[GBS_MAX_LANES] = {};
  hipEvent_t ev_fork = nullptr;
  hipEvent_t ev_join[GBS_MAX_LANES] = {};
  // timing
  bool timing = false;
  std::vector<EventPair> lf_ev, first_ev;
  size_t lf_used = 0, first_used = 0;
  // timing of the blocked adjoint's pass launches (one lane), with the
  // algorithmic bytes of the timed launches
  std::vector<EventPair> adj_ev;
  size_t adj_used = 0;
  double adj_bytes = 0;
};

namespace {

constexpr size_t kAlign = 256;
constexpr int kFourierMax = 8192;   // the Fourier derivative costs n^2 per evaluation
size_t align_up(size_t v) { return (v + kAlign - 1) / kAlign * kAlign; }

int fields_of(int op) {
  return op == GBS_ADVECT1D ? 1 : (op == GBS_ACOUSTIC2D ? 3 : (op == GBS_ACOUSTIC3D ? 4 : 0));
}
int dims_of(int op) { return op == GBS_ADVECT1D ? 1 : (op == GBS_ACOUSTIC2D ? 2 : 3); }
size_t dsize(int dtype) { return dtype == GBS_F32 ? 4 : 8; }

int validate_problem(const gbs_problem* p) {
  if (!p) return fail(GBS_EINVAL, "problem is null");
  if (!fields_of(p->op)) return fail(GBS_EINVAL, "unknown operator %d", p->op);
  if (p->fd_order == GBS_FD_SPECTRAL) {
    if (p->op != GBS_ADVECT1D)
      return fail(GBS_EUNSUPPORTED, "the Fourier derivative is built for GBS_ADVECT1D only");
    if (p->n[0] < 4 || p->n[0] > kFourierMax)
      return fail(GBS_EINVAL, "the Fourier derivative needs 4 <= n <= %d points", kFourierMax);
  } else if (p->fd_order != 4 && p->fd_order != 8) {
    return fail(GBS_EUNSUPPORTED, "fd_order must be 4, 8 or GBS_FD_SPECTRAL");
  }
  if (p->dtype != GBS_F32 && p->dtype != GBS_F64) return fail(GBS_EINVAL, "dtype must be F32 or F64");
  if (p->n_rhs < 1 || p->n_rhs > 65535) return fail(GBS_EINVAL, "n_rhs out of range");
  const int r = p->fd_order / 2;
  const int d = dims_of(p->op);
  for (int a = 0; a < 3; ++a) {
    if (a < d) {
      if (p->n[a] < 2 * r + 1 || p->n[a] > (1 << 30))
        return fail(GBS_EINVAL, "grid size along axis %d must be in [%d, 2^30]", a, 2 * r + 1);
    } else if (p->n[a] != 1) {
      return fail(GBS_EINVAL, "unused axis %d must have size 1", a);
    }
  }
  if (p->op != GBS_ADVECT1D) {
    if (p->c2_field) {
      if (!(p->c_max > 0) || !std::isfinite(p->c_max))
        return fail(GBS_EINVAL, "c_max must be given (> 0) with a coefficient field");
    } else if (!(p->c2 > 0) || !std::isfinite(p->c2)) {
      return fail(GBS_EINVAL, "constant c^2 must be positive and finite");
    }
  }
  return GBS_OK;
}

int validate_scheme(const gbs_scheme* s) {
  if (!s || !s->steps || !s->weights) return fail(GBS_EINVAL, "scheme or its arrays are null");
  if (s->k < 1 || s->k > GBS_MAX_SEQ) return fail(GBS_EINVAL, "k must be in [1, %d]", GBS_MAX_SEQ);
  if (s->p <= 0 || s->p % 2) return fail(GBS_EORDER, "order p must be a positive even integer");
  if (s->p % 4 == 2)
    return fail(GBS_EORDER, "order p = %d = 2 (mod 4): no imaginary-axis coverage", s->p);
  int st = check_steps(s->k, s->steps);
  if (st) return st;
  if (s->k < s->p / 2) return fail(GBS_ESTEPS, "k = %d sequences cannot reach order %d", s->k, s->p);
  // order constraints sum_j c_j N_j^(-2q) = [q == 0], checked to a tolerance
  // relative to sum_j |c_j| N_j^(-2q)
  for (int q = 0; q < s->p / 2; ++q) {
    long double sum = 0, mag = 0;
    for (int j = 0; j < s->k; ++j) {
      if (!std::isfinite(s->weights[j])) return fail(GBS_EINVAL, "weight %d is not finite", j);
      long double v = powl((long double)s->steps[j], -2.0L * q) * s->weights[j];
      sum += v;
      mag += fabsl(v);
    }
    long double want = q == 0 ? 1.0L : 0.0L;
    if (fabsl(sum - want) > 1e-12L * std::max(mag, 1e-300L))
      return fail(GBS_EORDER, "weights violate order constraint %d (residual %Lg)", q, sum - want);
  }
  return GBS_OK;
}

// levels per sequence: two for the streaming sweeps; the 2-D operator also
// has the temporally blocked passes, which read one pair of levels and
// write the other (and the FP64 y* into a free pair at the end)
int levels_per_seq(const gbs_problem* p) { return p->op == GBS_ACOUSTIC2D ? 4 : 2; }

constexpr size_t kSrcBytes = (GBS_MAX_SRC * sizeof(SrcDesc) + kAlign - 1) / kAlign * kAlign;
constexpr size_t kRecBytes = (GBS_MAX_REC * sizeof(RecDesc) + kAlign - 1) / kAlign * kAlign;

// b_1..b_K of the Fourier derivative, K = (n-1)/2 (fourier_dsum)
size_t fourier_bytes(const gbs_problem* p) {
  return p->fd_order == GBS_FD_SPECTRAL ? align_up((size_t)((p->n[0] - 1) / 2) * 8) : 0;
}

size_t workspace_bytes(const gbs_problem* p, int k) {
  const int64_t pts = p->n[0] * p->n[1] * p->n[2];
  const size_t elems = (size_t)p->n_rhs * fields_of(p->op) * pts;
  return kSrcBytes + kRecBytes + fourier_bytes(p) + align_up(elems * 8) +
         levels_per_seq(p) * (size_t)k * align_up(elems * dsize(p->dtype));
}

// App. A: the operator's eigenvalues (on the imaginary axis, modulus up to
// rho = c_max sigma sqrt(sum_a n_a^2)) must lie in the stability domain.
int check_stable(const gbs_problem* prob, const gbs_scheme* sch, double H) {
  if (prob->flags & GBS_FLAG_NO_STABILITY_CHECK) return GBS_OK;
  // The FP64 weights stand for an exact scheme: the free weights (those
  // beyond the first p/2 in the given order) as given, the dependent ones
  // re-solved exactly from the order constraints (Sect. 3.7).  Taken at their
  // binary values instead, rounding can leave sum_j c_j = 1 + 1 ulp, which
  // puts the origin itself outside the stability domain (ISB 0).  The
  // projection is used only if it moves no weight by more than 1e-12 of
  // sum |c| (otherwise the given weights are not an order-p scheme and are
  // checked as they are).
  const int k = sch->k, rows = sch->p / 2;
  std::vector<Rational> c(k);
  for (int j = 0; j < k; ++j) c[j] = Rational::from_double(sch->weights[j]);
  if (k >= rows && rows > 0) {
    std::vector<int32_t> fidx;
    std::vector<Rational> cf;
    for (int j = rows; j < k; ++j) {
      fidx.push_back(j);
      cf.push_back(c[j]);
    }
    std::vector<Rational> cp;
    const std::string saved = g_last_error;
    if (exact_weights(sch->p, k, sch->steps, k - rows, fidx.data(), cf.data(), cp) == GBS_OK) {
      double sum = 0, dev = 0;
      for (int j = 0; j < k; ++j) {
        sum += std::fabs(sch->weights[j]);
        dev = std::max(dev, std::fabs(cp[j].to_double() - sch->weights[j]));
      }
      if (dev <= 1e-12 * sum) c = cp;
    }
    g_last_error = saved;                            // a failed projection is no error
  }
  const double isb = isb_of(k, sch->steps, c);
  const int d = dims_of(prob->op);
  double s2 = 0;
  for (int a = 0; a < d; ++a) s2 += (double)prob->n[a] * (double)prob->n[a];
  const double cmax = prob->op == GBS_ADVECT1D
                          ? 1.0
                          : (prob->c2_field ? prob->c_max : std::sqrt(prob->c2));
  const double rho = cmax * stencil_sigma(prob->fd_order) * std::sqrt(s2);
  if (H * rho > isb)
    return fail(GBS_EUNSTABLE, "H * rho = %.6g exceeds the scheme's ISB %.6g", H * rho, isb);
  return GBS_OK;
}

// rho = c_max sigma sqrt(sum_a n_a^2): the operator's spectral radius bound
double rho_of(const gbs_problem* prob) {
  const int d = dims_of(prob->op);
  double s2 = 0;
  for (int a = 0; a < d; ++a) s2 += (double)prob->n[a] * (double)prob->n[a];
  const double cmax = prob->op == GBS_ADVECT1D
                          ? 1.0
                          : (prob->c2_field ? prob->c_max : std::sqrt(prob->c2));
  return cmax * stencil_sigma(prob->fd_order) * std::sqrt(s2);
}

// Weights b_1..b_K of the Fourier derivative as a centred difference over
// the whole period (fourier_dsum): b_k = pi (-1)^(k+1) cot(pi k / n) for even
// n, pi (-1)^(k+1) / sin(pi k / n) for odd n (the periodic differentiation
// matrix of the trigonometric interpolant, scaled to period 1).
void fourier_weights(gbs_plan* P) {
  const int64_t n = P->prob.n[0];
  const int K = (int)((n - 1) / 2);
  const double pi = 3.14159265358979323846;
  std::vector<double> b(K);
  for (int k = 1; k <= K; ++k) {
    const double t = pi * (double)k / (double)n;
    const double v = n % 2 == 0 ? std::cos(t) / std::sin(t) : 1.0 / std::sin(t);
    b[k - 1] = (k % 2 ? pi : -pi) * v;
  }
  if (P->prob.dtype == GBS_F64) {
    P->fourier_host.resize(b.size() * sizeof(double));
    std::memcpy(P->fourier_host.data(), b.data(), P->fourier_host.size());
  } else {
    std::vector<float> bf(b.begin(), b.end());
    P->fourier_host.resize(bf.size() * sizeof(float));
    std::memcpy(P->fourier_host.data(), bf.data(), P->fourier_host.size());
  }
}

// The Fourier weights reach the workspace on the plan's stream before the
// first step that reads them (plan creation itself makes no device call).
int upload_fourier(gbs_plan* P) {
  if (!P->fourier_dev || P->fourier_ready || P->fourier_host.empty()) return GBS_OK;
  if (hipMemcpyAsync(P->fourier_dev, P->fourier_host.data(), P->fourier_host.size(),
                     hipMemcpyHostToDevice, P->stream) != hipSuccess)
    return fail(GBS_EDEVICE, "copy of the Fourier-derivative weights failed");
  P->fourier_ready = true;
  return GBS_OK;
}

double ricker(double t, double f0, double delay) {
  const double pi = 3.14159265358979323846;
  const double a = (pi * f0 * (t - delay)) * (pi * f0 * (t - delay));
  return (1.0 - 2.0 * a) * std::exp(-a);
}

EventPair& next_event(std::vector<EventPair>& pool, size_t& used) {
  if (used == pool.size()) {
    EventPair e;
    hipEventCreate(&e.a);
    hipEventCreate(&e.b);
    pool.push_back(e);
  }
  return pool[used++];
}

template <typename T>
void fill_geometry(const gbs_plan* P, Geometry& g, T& c2c, const T*& c2f, T& ix, T& iy, T& iz) {
  g.nx = (int32_t)P->prob.n[0];
  g.ny = (int32_t)P->prob.n[1];
  g.nz = (int32_t)P->prob.n[2];
  g.nsrc = P->nsrc;
  g.field = P->field;
  g.state = P->state;
  g.fourier = P->fourier_dev;
  const double den = P->prob.fd_order == 8 ? 840.0 : 12.0;
  ix = (T)((double)P->prob.n[0] / den);
  iy = (T)((double)P->prob.n[1] / den);
  iz = (T)((double)P->prob.n[2] / den);
  c2c = (T)(P->prob.op == GBS_ADVECT1D ? 1.0 : P->prob.c2);
  c2f = (const T*)P->prob.c2_field;
}

int resolve_variant(const gbs_plan* P) {
  if (P->variant != GBS_VARIANT_AUTO) return P->variant;
  if (P->prob.op == GBS_ACOUSTIC2D) return GBS_VARIANT_TEMPORAL_S5;
  // the z-marching adjoint sweeps index a field with 32-bit element offsets
  if (P->prob.op == GBS_ACOUSTIC3D)
    return P->field < (int64_t(1) << 31) ? GBS_VARIANT_TILE3D : GBS_VARIANT_FLAT;
  return GBS_VARIANT_FLAT;
}

bool is_temporal(int v) {
  return (v >= GBS_VARIANT_TEMPORAL && v <= GBS_VARIANT_TEMPORAL_S6) ||
         v == GBS_VARIANT_TEMPORAL_WG4 || v == GBS_VARIANT_TEMPORAL_WG8;
}

// Shape of a temporally blocked variant: at most G evaluations per pass,
// time skew R (false) or R+1 (true), WPG wavefronts sharing edges.
struct TemporalShape {
  int G;
  bool skew1;
  int wpg;
};
TemporalShape temporal_shape(int v, int fd_order) {
  const int wpg = v == GBS_VARIANT_TEMPORAL_WG4 ? 4 : v == GBS_VARIANT_TEMPORAL_WG8 ? 8 : 1;
  if (fd_order == 8) return {3, true, wpg};
  switch (v) {
    case GBS_VARIANT_TEMPORAL4: return {4, false, 1};
    case GBS_VARIANT_TEMPORAL_S5: return {5, true, 1};
    case GBS_VARIANT_TEMPORAL_S6: return {6, true, 1};
    default: return {7, false, wpg};
  }
}

// Passes of every sequence: the N_j + 1 evaluations split into
// ceil((N_j+1)/G) passes of near-equal size; a sequence's pass q runs in
// round round0[j] + q.  Sequences with several passes start in round 0.
// With balance = true single-pass sequences go to the round with the least
// work so far (work of a pass ~ g times its halo overhead
// 64 wpg / (64 wpg - 2 g R)); otherwise they run in round 0, which measured
// faster on the 2048^2 workload (the first round's extra waves fill the GPU
// better than an even split).
struct PassSchedule {
  int npass[GBS_MAX_SEQ];
  int gsz[GBS_MAX_SEQ][32];
  int round0[GBS_MAX_SEQ];
  int nrounds = 0;
};

int make_schedule(const int32_t* steps, int k, int G, int R, int wpg, PassSchedule& s,
                  bool balance = false, int plus = 1) {
  double work[64] = {0};
  s.nrounds = 0;
  auto cost = [&](int g) { return g * (64.0 * wpg) / (64.0 * wpg - 2.0 * g * R); };
  for (int j = 0; j < k; ++j) {
    const int E = steps[j] + plus;                   // evaluations of sequence j
    const int np = (E + G - 1) / G;
    if (np > 32) return fail(GBS_EUNSUPPORTED, "too many passes per sequence");
    s.npass[j] = np;
    for (int q = 0; q < np; ++q) s.gsz[j][q] = E / np + (q < E % np ? 1 : 0);
    s.nrounds = std::max(s.nrounds, np);
  }
  for (int j = 0; j < k; ++j) {
    if (s.npass[j] > 1) {
      s.round0[j] = 0;
      for (int q = 0; q < s.npass[j]; ++q) work[q] += cost(s.gsz[j][q]);
    }
  }
  // single-pass sequences, largest first
  int ord[GBS_MAX_SEQ], n1 = 0;
  for (int j = 0; j < k; ++j)
    if (s.npass[j] == 1) ord[n1++] = j;
  std::sort(ord, ord + n1, [&](int a, int b) { return s.gsz[a][0] > s.gsz[b][0]; });
  for (int t = 0; t < n1; ++t) {
    const int j = ord[t];
    int best = 0;
    for (int r = 1; balance && r < s.nrounds; ++r)
      if (work[r] < work[best]) best = r;
    s.round0[j] = best;
    work[best] += cost(s.gsz[j][0]);
  }
  return GBS_OK;
}

// Wavefronts the current device holds at once for a pass kernel (occupancy
// x CUs), queried once per (device, kernel, block size).
template <typename K>
int resident_waves(K kernel, int block) {
  static std::mutex mu;
  static std::map<std::tuple<int, const void*, int>, int> cache;
  int dev = 0, cus = 0, per_cu = 0;
  if (hipGetDevice(&dev) != hipSuccess) return 0;
  const auto key = std::make_tuple(dev, (const void*)kernel, block);
  {
    std::lock_guard<std::mutex> lk(mu);
    auto it = cache.find(key);
    if (it != cache.end()) return it->second;
  }
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
      hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, block, 0) != hipSuccess ||
      per_cu < 1 || cus < 1)
    return 0;
  const int waves = per_cu * cus * (block / 64);
  std::lock_guard<std::mutex> lk(mu);
  cache[key] = waves;
  return waves;
}

// Rows per band of one round of passes when the plan leaves it automatic
// (band 0): the candidate minimising (rounds of resident wavefronts) x
// (rows one wavefront steps through, band + g (R + S)) for the round's
// largest g.  Few sequences in a round (its later rounds) get taller bands,
// so that the round does not end in a partly filled wave of wavefronts.
int band_for_round(const gbs_plan* P, int total_strips, int gmax, int R, int S, int slots) {
  if (P->band > 0) return P->band;
  const int ny = (int)P->prob.n[1];
  if (slots <= 0) return 64;
  const int cand[] = {32, 40, 48, 56, 64, 80, 96, 112, 128, 160, 192, 256};
  int best = 64;
  double best_t = 1e300;
  for (int b : cand) {
    const long waves = (long)total_strips * ((ny + b - 1) / b);
    const long rounds = (waves + slots - 1) / slots;
    const double t = (double)rounds * (double)(std::min(b, ny) + gmax * (R + S));
    if (t < best_t * (1.0 - 1e-9)) {
      best_t = t;
      best = b;
    }
  }
  return best;
}

// The tail kernel of the shared form: the last sequence's final pass with
// the combination (at most COMB_G evaluations).
constexpr int COMB_G = 4;

// How a temporally blocked macro step is organised: the pass schedule;
// whether f(t_0, y_0) is shared (one f0_march2d launch, first passes start
// from (y_0, y_1)); and whether the combination is folded into the last
// sequence's final pass, which needs that pass alone in the last round
// (every other y* is complete by then), at most COMB_G evaluations in it,
// at most COMB_MAX other sequences, one lane and no kept levels.
struct TemporalForm {
  PassSchedule sch;
  bool shared_f0 = true;
  bool fuse = false;
};

int temporal_form(const gbs_plan* P, int G, int R, int wpg, int order, TemporalForm& f) {
  f.shared_f0 = (P->form & GBS_FORM_SHARED_F0) != 0;
  int st = make_schedule(P->steps, P->k, G, R, wpg, f.sch, false, f.shared_f0 ? 0 : 1);
  if (st) return st;
  const PassSchedule& sch = f.sch;
  const int jl = P->order[P->k - 1];
  int last_round_seqs = 0;
  for (int j = 0; j < P->k; ++j)
    if (sch.round0[j] + sch.npass[j] == sch.nrounds) ++last_round_seqs;
  const int L = std::max(1, std::min(P->lanes, P->k));
  f.fuse = (P->form & GBS_FORM_FUSED_COMBINE) && order == 4 && wpg == 1 && L == 1 &&
           !P->keep_out && P->k >= 2 &&
           P->k - 1 <= COMB_MAX && last_round_seqs == 1 &&
           sch.round0[jl] + sch.npass[jl] == sch.nrounds &&
           sch.gsz[jl][sch.npass[jl] - 1] <= COMB_G;
  return GBS_OK;
}

template <typename T, int ORDER, int G, bool SKEW1, int WPG>
int run_temporal(gbs_plan* P, double t0, int n_macro, const T* yin, T* yout) {
  constexpr int R = Fd<ORDER>::R;
  // f(t_0, y_0) evaluated once per macro step (f0_march2d) and shared by the
  // first passes of all sequences, each of which then performs N_j
  // evaluations; F_0 lives in the plan's FP64 accumulator space
  TemporalForm form;
  int st = temporal_form(P, G, R, WPG, ORDER, form);
  if (st) return st;
  const PassSchedule& sch = form.sch;
  const bool shared_f0 = form.shared_f0;
  const bool fuse = form.fuse;
  const int* npass = sch.npass;
  PassArgs<T> pa;
  std::memset(&pa, 0, sizeof(pa));
  T c2c, invz;
  fill_geometry<T>(P, pa.g, c2c, pa.c2f, pa.invx, pa.invy, invz);
  pa.c2c = c2c;
  pa.src_dev = P->src_dev;
  pa.f0 = shared_f0 ? (const T*)P->acc : nullptr;
  F0Args<T> fa;
  std::memset(&fa, 0, sizeof(fa));
  fa.f0 = (T*)P->acc;
  fa.c2f = pa.c2f;
  fa.src = P->src_dev;
  fa.g = pa.g;
  fa.c2c = c2c;
  fa.invx = pa.invx;
  fa.invy = pa.invy;
  constexpr int F0_TY = 16;
  const unsigned f0_blocks =
      (unsigned)(((P->prob.n[0] + 63) / 64) * ((P->prob.n[1] + 4 * F0_TY - 1) / (4 * F0_TY)));
  const int nx = (int)P->prob.n[0];
  constexpr int S = SKEW1 ? R + 1 : R;
  const int slots_c = resident_waves(pass2d<T, ORDER, G, SKEW1, WPG, false>,
                                            WPG > 1 ? 64 * WPG : 256);
  const int slots_v = resident_waves(pass2d<T, ORDER, G, SKEW1, WPG, true>,
                                            WPG > 1 ? 64 * WPG : 256);
  const int slots = (P->prob.c2_field ? slots_v : slots_c) / WPG;   // units of WPG wavefronts
  CombineArgs<T> ca;
  std::memset(&ca, 0, sizeof(ca));
  ca.k = P->k;
  ca.n = (int64_t)P->prob.n_rhs * P->state;
  ca.yout = yout;
  for (int r = 0; r < P->k; ++r) {
    const int j = P->order[r];
    ca.c[r] = P->w[j];
    ca.ystar[r] = (const double*)P->pair[j][(npass[j] - 1) % 2 == 0 ? 0 : 1][0];
  }
  // lanes: sequences folded in pairs by ascending N (longest with shortest,
  // as the paper folds sequences onto cores, Sect. 3.6), pair i on lane
  // i mod L; each lane runs its passes on its own stream
  const int L = std::max(1, std::min(P->lanes, P->k));
  int lane_of[GBS_MAX_SEQ];
  for (int r = 0; r < P->k; ++r) lane_of[r] = std::min(r, P->k - 1 - r) % L;
  const int lane_slots = std::max(1, slots / L);
  // the combination folded into the last sequence's final pass (see
  // temporal_form)
  if (fuse) {
    for (int r = 0; r + 1 < P->k; ++r) {
      pa.comb.ystar[r] = ca.ystar[r];
      pa.comb.c[r] = ca.c[r];
    }
    pa.comb.n = P->k - 1;
    pa.comb.c_last = ca.c[P->k - 1];
    pa.comb.yout = yout;
  }
  const int slots_comb =
      fuse ? (P->prob.c2_field
                  ? resident_waves(pass2d<T, ORDER, COMB_G, true, 1, true, false, true>, 256)
                  : resident_waves(pass2d<T, ORDER, COMB_G, true, 1, false, false, true>, 256))
           : 0;
  for (int m = 0; m < n_macro; ++m) {
    const double t = t0 + m * P->H;
    const T* y0 = m == 0 ? yin : yout;
    if (shared_f0) {
      fa.y0 = y0;
      fa.amp = P->nsrc ? ricker(t, P->f0, P->delay) : 0.0;
      EventPair* ev = nullptr;
      if (P->timing) {
        ev = &next_event(P->first_ev, P->first_used);
        hipEventRecord(ev->a, P->stream);
      }
      hipLaunchKernelGGL((f0_march2d<T, ORDER, F0_TY>), dim3(f0_blocks, 1, P->prob.n_rhs),
                         dim3(256), 0, P->stream, fa);
      if (ev) hipEventRecord(ev->b, P->stream);
    }
    if (L > 1) {
      hipEventRecord(P->ev_fork, P->stream);
      for (int l = 1; l < L; ++l) hipStreamWaitEvent(P->lane_stream[l], P->ev_fork, 0);
    }
    for (int l = 0; l < L; ++l)
    for (int rr = 0; rr < sch.nrounds; ++rr) {
      hipStream_t ls = l == 0 ? P->stream : P->lane_stream[l];
      int n = 0, maxs = 0;
      for (int r = 0; r < P->k; ++r) {
        const int j = P->order[r];
        const int q = rr - sch.round0[j];
        if (lane_of[r] != l || q < 0 || q >= npass[j]) continue;
        PassSeq<T>& d = pa.seq[n++];
        d.hs = 0;
        const double h = P->H / P->steps[j];
        // the pass's input level is y_{s0}: s0 = evaluations so far (the
        // shared form's first pass starts from the pair (y_0, y_1))
        int s0 = shared_f0 ? 1 : 0;
        for (int qq = 0; qq < q; ++qq) s0 += sch.gsz[j][qq];
        d.g = sch.gsz[j][q];
        d.h = (T)h;
        d.flags = (q == 0 ? (shared_f0 ? PASS_F0 : PASS_FIRST) : 0) |
                  (q == npass[j] - 1 ? PASS_FINAL : 0);
        if (fuse && rr == sch.nrounds - 1) d.flags |= PASS_COMBINE;
        d.cur = q == 0 ? y0 : (const T*)P->pair[j][(q - 1) % 2][1];
        d.old = q == 0 ? (shared_f0 ? y0 : nullptr) : (const T*)P->pair[j][(q - 1) % 2][0];
        d.out_a = (T*)P->pair[j][q % 2][0];
        d.out_b = (T*)P->pair[j][q % 2][1];
        d.ystar = (double*)P->pair[j][q % 2][0];
        if (P->keep_out && q == npass[j] - 1) {
          // [macro step][sequence j][y_{N-1}, y_N][whole state]
          T* kb = (T*)P->keep_out + ((size_t)m * P->k + j) * 2 * ca.n;
          d.flags |= PASS_KEEP;
          d.out_a = kb;
          d.out_b = kb + ca.n;
        }
        d.strips = (nx + (64 * WPG - 2 * d.g * R) - 1) / (64 * WPG - 2 * d.g * R);
        for (int e = 0; e < d.g; ++e)
          d.amp[e] = P->nsrc ? ricker(t + (s0 + e) * h, P->f0, P->delay) : 0.0;
        maxs = std::max(maxs, d.strips);
      }
      if (n == 0) continue;
      // GBS_FORM_ALIGNED_FIRST: the first passes (all reading y_0) take the
      // strip geometry of the widest halo among them, so that workgroup u of
      // every sequence covers the same columns, and run in the grouped
      // order below, so that those workgroups meet on one XCD and read the
      // y_0 rows once from HBM
      const bool aligned = WPG == 1 && n > 1 && (P->form & GBS_FORM_ALIGNED_FIRST) && rr == 0;
      if (aligned) {
        int gmax = 0;
        for (int i = 0; i < n; ++i) gmax = std::max(gmax, pa.seq[i].g);
        const int wv = 64 - 2 * gmax * R;
        maxs = (nx + wv - 1) / wv;
        for (int i = 0; i < n; ++i) {
          pa.seq[i].hs = gmax * R;
          pa.seq[i].strips = maxs;
        }
      }
      pa.max_strips = maxs;
      {
        int strips = 0, gmax = 0;
        for (int i = 0; i < n; ++i) {
          strips += pa.seq[i].strips;
          gmax = std::max(gmax, pa.seq[i].g);
        }
        const bool tail = fuse && rr == sch.nrounds - 1;
        pa.band = band_for_round(P, strips, gmax, R, tail ? R + 1 : S,
                                 tail ? slots_comb : (L > 1 ? lane_slots : slots));
        pa.nbands = (int)((P->prob.n[1] + pa.band - 1) / pa.band);
      }
      const unsigned waves = (unsigned)maxs * pa.nbands;
      EventPair* ev = nullptr;
      if (P->timing) {
        ev = &next_event(P->lf_ev, P->lf_used);
        hipEventRecord(ev->a, ls);
      }
      const unsigned blocks = WPG > 1 ? waves : (waves + 3) / 4;
      dim3 grid(blocks, n, P->prob.n_rhs);
      const dim3 blk(WPG > 1 ? 64 * WPG : 256);
      pa.order = WPG == 1 && n > 1 ? (aligned && !P->wave_order ? 2 : P->wave_order) : 0;
      if (pa.order) {
        // sequences of one group of 4 units adjacent on one XCD
        pa.nseq = n;
        pa.per = (int)((blocks + 7) / 8);
        grid = dim3(8u * (unsigned)pa.per * (unsigned)n, 1, P->prob.n_rhs);
      }
      if constexpr (ORDER == 4 && WPG == 1) {
        if (fuse && rr == sch.nrounds - 1) {
          // the last sequence's final pass, forming y_out
          if (P->prob.c2_field)
            hipLaunchKernelGGL((pass2d<T, ORDER, COMB_G, true, 1, true, false, true>), grid, blk,
                               0, ls, pa);
          else
            hipLaunchKernelGGL((pass2d<T, ORDER, COMB_G, true, 1, false, false, true>), grid, blk,
                               0, ls, pa);
          if (ev) hipEventRecord(ev->b, ls);
          continue;
        }
      }
      // the kept-pairs stores live in their own instantiations so that the
      // plain forward kernels keep their register budget
      if constexpr (ORDER == 4) {
        if (P->keep_out) {
          if (P->prob.c2_field)
            hipLaunchKernelGGL((pass2d<T, ORDER, G, SKEW1, WPG, true, true>), grid, blk, 0, ls, pa);
          else
            hipLaunchKernelGGL((pass2d<T, ORDER, G, SKEW1, WPG, false, true>), grid, blk, 0, ls, pa);
          if (ev) hipEventRecord(ev->b, ls);
          continue;
        }
      }
      if (P->prob.c2_field)
        hipLaunchKernelGGL((pass2d<T, ORDER, G, SKEW1, WPG, true>), grid, blk, 0, ls, pa);
      else
        hipLaunchKernelGGL((pass2d<T, ORDER, G, SKEW1, WPG, false>), grid, blk, 0, ls, pa);
      if (ev) hipEventRecord(ev->b, ls);
    }
    if (L > 1) {
      for (int l = 1; l < L; ++l) {
        hipEventRecord(P->ev_join[l], P->lane_stream[l]);
        hipStreamWaitEvent(P->stream, P->ev_join[l], 0);
      }
    }
    if (fuse) continue;     // the last pass has formed y_out
    EventPair* ev = nullptr;
    if (P->timing) {
      ev = &next_event(P->first_ev, P->first_used);
      hipEventRecord(ev->a, P->stream);
    }
    hipLaunchKernelGGL((combine_kernel<T>), dim3((unsigned)((ca.n + 255) / 256)), dim3(256), 0,
                       P->stream, ca);
    if (ev) hipEventRecord(ev->b, P->stream);
  }
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return fail(GBS_EDEVICE, "kernel launch failed: %s", hipGetErrorString(e));
  return GBS_OK;
}

template <typename T, int ORDER, int TY, bool NT>
void launch_march2d(gbs_plan* P, const StepArgs<T>& sa, int n, unsigned gz) {
  const int ntx = (int)((P->prob.n[0] + 63) / 64);
  const int nty = (int)((P->prob.n[1] + 4 * TY - 1) / (4 * TY));
  hipLaunchKernelGGL((lf_march2d<T, ORDER, TY, NT>), dim3(ntx * nty, n, gz), dim3(256), 0,
                     P->stream, sa);
}

template <typename T, int ORDER, int TZ>
void launch_march3d(gbs_plan* P, const StepArgs<T>& sa, int n, unsigned gz) {
  const int ntx = (int)((P->prob.n[0] + 63) / 64);
  const int nty = (int)((P->prob.n[1] + 3) / 4);
  const int ntz = (int)((P->prob.n[2] + TZ - 1) / TZ);
  hipLaunchKernelGGL((lf_march3d<T, ORDER, TZ, false>), dim3(ntx * nty * ntz, n, gz), dim3(256),
                     0, P->stream, sa);
}

// LDS-tiled 3-D sweeps: 64 x 16 columns per 1024-thread block, at most
// TILE_TZ planes per block
constexpr int TILE_TZ = 128;

unsigned tile3d_blocks(const gbs_plan* P, int tz) {
  const int ntx = (int)((P->prob.n[0] + 63) / 64);
  const int nty = (int)((P->prob.n[1] + 15) / 16);
  const int ntz = (int)((P->prob.n[2] + tz - 1) / tz);
  return (unsigned)(ntx * nty * ntz);
}

// Planes per block of an LDS-tiled sweep launch with `mult` blocks per tile
// (sequences x right-hand sides): its blocks run in rounds of the blocks the
// GPU holds at once, so the chunking (at most TILE_TZ planes) is the one that
// minimises rounds x (planes + the 2R warm-up planes of a chunk).  A launch
// of many blocks keeps TILE_TZ; one of a few rounds (one sequence, few
// right-hand sides) gets shorter chunks so that its last round is not
// mostly idle.
template <int ORDER, typename K>
int tile3d_planes(const gbs_plan* P, K kernel, long mult) {
  constexpr int R = Fd<ORDER>::R;
  const long txy = (long)((P->prob.n[0] + 63) / 64) * (long)((P->prob.n[1] + 15) / 16);
  const int nz = (int)P->prob.n[2];
  const long slots = std::max(1, resident_waves(kernel, 1024) / 16);
  int best_tz = std::min(TILE_TZ, nz), prev = 0;
  double best = 1e300;
  for (int m = (nz + TILE_TZ - 1) / TILE_TZ; m <= std::max(1, nz / 16); ++m) {
    const int tz = (nz + m - 1) / m;
    if (tz == prev) continue;
    prev = tz;
    const long blocks = txy * ((nz + tz - 1) / tz) * mult;
    const double cost = (double)((blocks + slots - 1) / slots) * (double)(tz + 2 * R);
    if (cost < best * (1.0 - 1e-9)) {
      best = cost;
      best_tz = tz;
    }
  }
  return best_tz;
}

template <typename T, int ORDER, int OP>
void launch_first(gbs_plan* P, const FirstArgs<T>& fa, unsigned gx, unsigned gz) {
  if constexpr (OP == OP_AC3D && ORDER != GBS_FD_SPECTRAL) {
    if (resolve_variant(P) == GBS_VARIANT_TILE3D) {
      FirstArgs<T> a = fa;
      a.tz = tile3d_planes<ORDER>(P, first_tile3d<T, ORDER, TILE_TZ>, (long)gz);
      hipLaunchKernelGGL((first_tile3d<T, ORDER, TILE_TZ>), dim3(tile3d_blocks(P, a.tz), 1, gz),
                         dim3(1024), 0, P->stream, a);
      return;
    }
  }
  if constexpr (OP == OP_AC3D) {
    const int v = resolve_variant(P);
    if (v == GBS_VARIANT_MARCH8 || v == GBS_VARIANT_MARCH16) {
      const int ntx = (int)((P->prob.n[0] + 63) / 64);
      const int nty = (int)((P->prob.n[1] + 3) / 4);
      const int ntz = (int)((P->prob.n[2] + 63) / 64);
      hipLaunchKernelGGL((first_march3d<T, ORDER, 64>), dim3(ntx * nty * ntz, 1, gz), dim3(256), 0,
                         P->stream, fa);
      return;
    }
  }
  hipLaunchKernelGGL((first_kernel<T, ORDER, OP>), dim3(gx, 1, gz), dim3(256), 0, P->stream, fa);
}

template <typename T, int ORDER, int OP>
void launch_lf(gbs_plan* P, const StepArgs<T>& sa, int n, unsigned gx, unsigned gz) {
  if constexpr (OP == OP_AC3D && ORDER != GBS_FD_SPECTRAL) {
    if (resolve_variant(P) == GBS_VARIANT_TILE3D) {
      StepArgs<T> a = sa;
      a.tz = tile3d_planes<ORDER>(P, lf_tile3d<T, ORDER, TILE_TZ>, (long)n * gz);
      hipLaunchKernelGGL((lf_tile3d<T, ORDER, TILE_TZ>), dim3(tile3d_blocks(P, a.tz) * n, 1, gz),
                         dim3(1024), 0, P->stream, a);
      return;
    }
  }
  if constexpr (OP == OP_AC3D) {
    switch (resolve_variant(P)) {
      case GBS_VARIANT_MARCH8: launch_march3d<T, ORDER, 64>(P, sa, n, gz); return;
      case GBS_VARIANT_MARCH16: launch_march3d<T, ORDER, 128>(P, sa, n, gz); return;
      default: break;
    }
  }
  if constexpr (OP == OP_AC2D) {
    switch (resolve_variant(P)) {
      case GBS_VARIANT_MARCH8: launch_march2d<T, ORDER, 8, false>(P, sa, n, gz); return;
      case GBS_VARIANT_MARCH16: launch_march2d<T, ORDER, 16, false>(P, sa, n, gz); return;
      case GBS_VARIANT_MARCH8_NT: launch_march2d<T, ORDER, 8, true>(P, sa, n, gz); return;
      case GBS_VARIANT_MARCH16_NT: launch_march2d<T, ORDER, 16, true>(P, sa, n, gz); return;
      default: break;
    }
  }
  if (resolve_variant(P) == GBS_VARIANT_PLAIN) {
    // one launch per sequence: the unfused reference form
    StepArgs<T> one = sa;
    for (int i = 0; i < n; ++i) {
      one.seq[0] = sa.seq[i];
      hipLaunchKernelGGL((lf_kernel<T, ORDER, OP>), dim3(gx, 1, gz), dim3(256), 0, P->stream, one);
    }
    return;
  }
  hipLaunchKernelGGL((lf_kernel<T, ORDER, OP>), dim3(gx, n, gz), dim3(256), 0, P->stream, sa);
}

template <typename T, int ORDER, int OP>
int run(gbs_plan* P, double t0, int n_macro, const T* yin, T* yout) {
  const int block = 256;
  const unsigned gx =
      (unsigned)((P->field * PointLanes<ORDER>::L + block - 1) / block);
  const unsigned gz = (unsigned)P->prob.n_rhs;
  FirstArgs<T> fa;
  StepArgs<T> sa;
  std::memset(&fa, 0, sizeof(fa));
  std::memset(&sa, 0, sizeof(sa));
  fill_geometry<T>(P, fa.g, fa.c2c, fa.c2f, fa.invx, fa.invy, fa.invz);
  fill_geometry<T>(P, sa.g, sa.c2c, sa.c2f, sa.invx, sa.invy, sa.invz);
  std::memcpy(fa.src, P->src, sizeof(P->src));
  std::memcpy(sa.src, P->src, sizeof(P->src));
  sa.acc = P->acc;
  sa.yout = yout;
  fa.nseq = P->k;
  for (int j = 0; j < P->k; ++j) {
    fa.out[j] = (T*)P->lev[j][1];
    fa.h[j] = (T)(P->H / P->steps[j]);
  }
  for (int m = 0; m < n_macro; ++m) {
    const double t = t0 + m * P->H;
    const T* src = m == 0 ? yin : yout;
    fa.y0 = src;
    fa.amp = P->nsrc ? ricker(t, P->f0, P->delay) : 0.0;
    EventPair* ev = nullptr;
    if (P->timing) {
      ev = &next_event(P->first_ev, P->first_used);
      hipEventRecord(ev->a, P->stream);
    }
    launch_first<T, ORDER, OP>(P, fa, gx, gz);
    if (ev) hipEventRecord(ev->b, P->stream);
    for (int s = 1; s <= P->nmax; ++s) {
      int n = 0;
      for (int r = 0; r < P->k; ++r) {
        const int j = P->order[r];
        const int N = P->steps[j];
        if (N < s) continue;
        const double h = P->H / N;
        SeqDesc<T>& d = sa.seq[n++];
        d.cur = (const T*)P->lev[j][s & 1];
        d.old = s == 1 ? src : (const T*)P->lev[j][1 - (s & 1)];
        d.out = (T*)P->lev[j][1 - (s & 1)];
        d.h2 = (T)(2.0 * h);
        d.cw = P->w[j];
        d.amp = P->nsrc ? ricker(t + s * h, P->f0, P->delay) : 0.0;
        d.mode = 0;
        if (s == N) {
          d.mode |= MODE_LAST;
          if (r == 0) d.mode |= MODE_FIRST;
          if (r == P->k - 1) d.mode |= MODE_FINAL;
        }
      }
      ev = nullptr;
      if (P->timing) {
        ev = &next_event(P->lf_ev, P->lf_used);
        hipEventRecord(ev->a, P->stream);
      }
      launch_lf<T, ORDER, OP>(P, sa, n, gx, gz);
      if (ev) hipEventRecord(ev->b, P->stream);
    }
  }
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return fail(GBS_EDEVICE, "kernel launch failed: %s", hipGetErrorString(e));
  return GBS_OK;
}

template <typename T, int ORDER, int OP>
int run_rk4(gbs_plan* P, double t0, int n_steps, double h, const T* yin, T* yout) {
  RK4Args<T> ra;
  std::memset(&ra, 0, sizeof(ra));
  fill_geometry<T>(P, ra.g, ra.c2c, ra.c2f, ra.invx, ra.invy, ra.invz);
  std::memcpy(ra.src, P->src, sizeof(P->src));
  ra.acc = P->acc;
  ra.h = h;
  T* st[2] = {(T*)P->lev[0][0], (T*)P->lev[0][1]};
  const unsigned gx = (unsigned)((P->field * PointLanes<ORDER>::L + 255) / 256);
  const unsigned gz = (unsigned)P->prob.n_rhs;
  const double frac[4] = {0.0, 0.5, 0.5, 1.0};
  for (int m = 0; m < n_steps; ++m) {
    const double t = t0 + m * h;
    ra.yn = m == 0 ? yin : yout;
    for (int s = 0; s < 4; ++s) {
      ra.stage = s;
      ra.ys = s == 0 ? ra.yn : st[(s - 1) % 2];
      ra.out = s == 3 ? yout : st[s % 2];
      ra.amp = P->nsrc ? ricker(t + frac[s] * h, P->f0, P->delay) : 0.0;
      hipLaunchKernelGGL((rk4_stage<T, ORDER, OP>), dim3(gx, 1, gz), dim3(256), 0, P->stream, ra);
    }
  }
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return fail(GBS_EDEVICE, "kernel launch failed: %s", hipGetErrorString(e));
  return GBS_OK;
}

template <typename T>
int dispatch_rk4(gbs_plan* P, double t0, int n, double h, const void* yin, void* yout) {
  const T* a = (const T*)yin;
  T* b = (T*)yout;
  const int op = P->prob.op;
  if (P->prob.fd_order == GBS_FD_SPECTRAL)
    return run_rk4<T, GBS_FD_SPECTRAL, OP_ADV1D>(P, t0, n, h, a, b);
  if (P->prob.fd_order == 4) {
    if (op == GBS_ADVECT1D) return run_rk4<T, 4, OP_ADV1D>(P, t0, n, h, a, b);
    if (op == GBS_ACOUSTIC2D) return run_rk4<T, 4, OP_AC2D>(P, t0, n, h, a, b);
    return run_rk4<T, 4, OP_AC3D>(P, t0, n, h, a, b);
  }
  if (op == GBS_ADVECT1D) return run_rk4<T, 8, OP_ADV1D>(P, t0, n, h, a, b);
  if (op == GBS_ACOUSTIC2D) return run_rk4<T, 8, OP_AC2D>(P, t0, n, h, a, b);
  return run_rk4<T, 8, OP_AC3D>(P, t0, n, h, a, b);
}

template <typename T>
int dispatch_order(gbs_plan* P, double t0, int n, const void* yin, void* yout) {
  const T* a = (const T*)yin;
  T* b = (T*)yout;
  const int op = P->prob.op;
  const int v = resolve_variant(P);
  if (op == GBS_ACOUSTIC2D && is_temporal(v)) {
    if (P->prob.fd_order == 8) {
      if (v == GBS_VARIANT_TEMPORAL_WG4) return run_temporal<T, 8, 3, true, 4>(P, t0, n, a, b);
      if (v == GBS_VARIANT_TEMPORAL_WG8) return run_temporal<T, 8, 3, true, 8>(P, t0, n, a, b);
      return run_temporal<T, 8, 3, true, 1>(P, t0, n, a, b);
    }
    switch (v) {
      case GBS_VARIANT_TEMPORAL4: return run_temporal<T, 4, 4, false, 1>(P, t0, n, a, b);
      case GBS_VARIANT_TEMPORAL_S5: return run_temporal<T, 4, 5, true, 1>(P, t0, n, a, b);
      case GBS_VARIANT_TEMPORAL_S6: return run_temporal<T, 4, 6, true, 1>(P, t0, n, a, b);
      case GBS_VARIANT_TEMPORAL_WG4: return run_temporal<T, 4, 7, false, 4>(P, t0, n, a, b);
      case GBS_VARIANT_TEMPORAL_WG8: return run_temporal<T, 4, 7, false, 8>(P, t0, n, a, b);
      default: return run_temporal<T, 4, 7, false, 1>(P, t0, n, a, b);
    }
  }
  if (P->prob.fd_order == GBS_FD_SPECTRAL) return run<T, GBS_FD_SPECTRAL, OP_ADV1D>(P, t0, n, a, b);
  if (P->prob.fd_order == 4) {
    if (op == GBS_ADVECT1D) return run<T, 4, OP_ADV1D>(P, t0, n, a, b);
    if (op == GBS_ACOUSTIC2D) return run<T, 4, OP_AC2D>(P, t0, n, a, b);
    return run<T, 4, OP_AC3D>(P, t0, n, a, b);
  }
  if (op == GBS_ADVECT1D) return run<T, 8, OP_ADV1D>(P, t0, n, a, b);
  if (op == GBS_ACOUSTIC2D) return run<T, 8, OP_AC2D>(P, t0, n, a, b);
  return run<T, 8, OP_AC3D>(P, t0, n, a, b);
}

}  // namespace

extern "C" int gbs_plan_workspace_bytes(const gbs_problem* prob, const gbs_scheme* sch,
                                        size_t* bytes) {
  int st = validate_problem(prob);
  if (st) return st;
  if (!sch || !bytes) return fail(GBS_EINVAL, "null argument");
  if (sch->k < 1 || sch->k > GBS_MAX_SEQ) return fail(GBS_EINVAL, "k out of range");
  *bytes = workspace_bytes(prob, sch->k);
  return GBS_OK;
}

namespace {

// Validates the problem and scheme and sets up *P (a default-constructed
// plan) on the caller's workspace.
int plan_init(gbs_plan* P, const gbs_problem* prob, const gbs_scheme* sch, double H,
              void* workspace, size_t ws_bytes, void* hip_stream) {
  try {
    int st = validate_problem(prob);
    if (st) return st;
    st = validate_scheme(sch);
    if (st) return st;
    if (!(H > 0) || !std::isfinite(H)) return fail(GBS_EINVAL, "H must be positive and finite");
    if (!workspace) return fail(GBS_EINVAL, "workspace is null");
    if ((uintptr_t)workspace % kAlign) return fail(GBS_EINVAL, "workspace must be 256-byte aligned");
    const size_t need = workspace_bytes(prob, sch->k);
    if (ws_bytes < need)
      return fail(GBS_ENOMEM, "workspace has %zu bytes, needs %zu", ws_bytes, need);
    st = check_stable(prob, sch, H);
    if (st) return st;
    P->prob = *prob;
    P->k = sch->k;
    for (int j = 0; j < sch->k; ++j) {
      P->steps[j] = sch->steps[j];
      P->w[j] = sch->weights[j];
      P->order[j] = j;
      P->nmax = std::max(P->nmax, (int)sch->steps[j]);
    }
    std::sort(P->order, P->order + P->k, [&](int a, int b) { return P->steps[a] < P->steps[b]; });
    P->H = H;
    P->F = fields_of(prob->op);
    P->field = prob->n[0] * prob->n[1] * prob->n[2];
    P->state = P->F * P->field;
    P->stream = (hipStream_t)hip_stream;
    const size_t elems = (size_t)prob->n_rhs * P->state;
    char* base = (char*)workspace;
    P->src_dev = (SrcDesc*)base;
    base += kSrcBytes;
    P->rec_dev = (RecDesc*)base;
    base += kRecBytes;
    if (prob->fd_order == GBS_FD_SPECTRAL) {
      fourier_weights(P);
      P->fourier_dev = base;
      base += fourier_bytes(prob);
    }
    P->acc = (double*)base;
    base += align_up(elems * 8);
    const size_t lb = align_up(elems * dsize(prob->dtype));
    for (int j = 0; j < P->k; ++j) {
      char* sb = base + (size_t)j * levels_per_seq(prob) * lb;
      P->lev[j][0] = sb;
      P->lev[j][1] = sb + lb;
      if (levels_per_seq(prob) == 4)
        for (int q = 0; q < 2; ++q)
          for (int l = 0; l < 2; ++l) P->pair[j][q][l] = sb + (2 * q + l) * lb;
    }
    return GBS_OK;
  } catch (const std::exception& e) {
    return fail(GBS_EINVAL, "gbs_plan_create: %s", e.what());
  }
}

}  // namespace

extern "C" int gbs_plan_create(gbs_plan** out, const gbs_problem* prob, const gbs_scheme* sch,
                               double H, void* workspace, size_t ws_bytes, void* hip_stream) {
  if (!out) return fail(GBS_EINVAL, "out is null");
  *out = nullptr;
  gbs_plan* P = new (std::nothrow) gbs_plan();
  if (!P) return fail(GBS_ENOMEM, "out of host memory");
  const int st = plan_init(P, prob, sch, H, workspace, ws_bytes, hip_stream);
  if (st) {
    delete P;
    return st;
  }
  *out = P;
  return GBS_OK;
}

extern "C" int gbs_plan_set_sources(gbs_plan* P, int32_t n_src, const int32_t* rhs,
                                    const int64_t* flat_index, const double* weight, double f0,
                                    double delay) {
  if (!P) return fail(GBS_EINVAL, "plan is null");
  if (n_src < 0 || n_src > GBS_MAX_SRC) return fail(GBS_EINVAL, "n_src out of range");
  if (n_src && P->prob.op == GBS_ADVECT1D) return fail(GBS_EINVAL, "sources need an acoustic plan");
  if (n_src && (!rhs || !flat_index || !weight)) return fail(GBS_EINVAL, "source arrays are null");
  if (n_src && !(f0 > 0)) return fail(GBS_EINVAL, "f0 must be positive");
  for (int s = 0; s < n_src; ++s) {
    if (rhs[s] < 0 || rhs[s] >= P->prob.n_rhs) return fail(GBS_EINVAL, "source %d: rhs out of range", s);
    if (flat_index[s] < 0 || flat_index[s] >= P->field)
      return fail(GBS_EINVAL, "source %d: index out of range", s);
    if (!std::isfinite(weight[s])) return fail(GBS_EINVAL, "source %d: weight not finite", s);
  }
  std::memset(P->src, 0, sizeof(P->src));
  for (int s = 0; s < n_src; ++s) {
    P->src[s].idx = flat_index[s];
    P->src[s].w = weight[s];
    P->src[s].rhs = rhs[s];
  }
  if (hipMemcpyAsync(P->src_dev, P->src, sizeof(P->src), hipMemcpyHostToDevice, P->stream) !=
          hipSuccess ||
      hipStreamSynchronize(P->stream) != hipSuccess)
    return fail(GBS_EDEVICE, "copying the sources to the workspace failed");
  P->nsrc = n_src;
  P->f0 = f0;
  P->delay = delay;
  return GBS_OK;
}

extern "C" int gbs_step(gbs_plan* P, double t0, int32_t n_macro, const void* y_in, void* y_out) {
  if (!P || !y_in || !y_out) return fail(GBS_EINVAL, "null argument");
  if (n_macro < 0) return fail(GBS_EINVAL, "n_macro must be >= 0");
  if (!std::isfinite(t0)) return fail(GBS_EINVAL, "t0 must be finite");
  if (n_macro == 0) {
    if (y_in != y_out) {
      const size_t bytes = (size_t)P->prob.n_rhs * P->state * dsize(P->prob.dtype);
      if (hipMemcpyAsync(y_out, y_in, bytes, hipMemcpyDeviceToDevice, P->stream) != hipSuccess)
        return fail(GBS_EDEVICE, "copy failed");
    }
    return GBS_OK;
  }
  const int up = upload_fourier(P);
  if (up) return up;
  if (P->prob.dtype == GBS_F64) return dispatch_order<double>(P, t0, n_macro, y_in, y_out);
  return dispatch_order<float>(P, t0, n_macro, y_in, y_out);
}

extern "C" int gbs_rk4_step(gbs_plan* P, double t0, int32_t n_steps, double h, const void* y_in,
                            void* y_out) {
  if (!P || !y_in || !y_out) return fail(GBS_EINVAL, "null argument");
  if (n_steps < 0) return fail(GBS_EINVAL, "n_steps must be >= 0");
  if (!std::isfinite(t0) || !(h > 0) || !std::isfinite(h))
    return fail(GBS_EINVAL, "t0 must be finite and h positive");
  if (!(P->prob.flags & GBS_FLAG_NO_STABILITY_CHECK)) {
    const double isb = 2.0 * std::sqrt(2.0);           // App. A: RK4's imaginary boundary
    const double hr = h * rho_of(&P->prob);
    if (hr > isb) return fail(GBS_EUNSTABLE, "h * rho = %.6g exceeds RK4's ISB 2 sqrt 2", hr);
  }
  if (n_steps == 0) {
    if (y_in != y_out) {
      const size_t bytes = (size_t)P->prob.n_rhs * P->state * dsize(P->prob.dtype);
      if (hipMemcpyAsync(y_out, y_in, bytes, hipMemcpyDeviceToDevice, P->stream) != hipSuccess)
        return fail(GBS_EDEVICE, "copy failed");
    }
    return GBS_OK;
  }
  const int up = upload_fourier(P);
  if (up) return up;
  if (P->prob.dtype == GBS_F64) return dispatch_rk4<double>(P, t0, n_steps, h, y_in, y_out);
  return dispatch_rk4<float>(P, t0, n_steps, h, y_in, y_out);
}

extern "C" int gbs_plan_set_variant(gbs_plan* P, int32_t variant) {
  if (!P) return fail(GBS_EINVAL, "plan is null");
  if (variant < GBS_VARIANT_AUTO || variant > GBS_VARIANT_TILE3D)
    return fail(GBS_EINVAL, "unknown variant %d", variant);
  if (variant == GBS_VARIANT_TILE3D && P->prob.op != GBS_ACOUSTIC3D)
    return fail(GBS_EUNSUPPORTED, "GBS_VARIANT_TILE3D is built for the 3-D operator only");
  const bool march3d = P->prob.op == GBS_ACOUSTIC3D &&
                       (variant == GBS_VARIANT_MARCH8 || variant == GBS_VARIANT_MARCH16 ||
                        variant == GBS_VARIANT_TILE3D);
  if (march3d && P->field >= (int64_t(1) << 31))
    return fail(GBS_EUNSUPPORTED, "the 3-D marching kernels need fields of fewer than 2^31 points");
  if (variant >= GBS_VARIANT_MARCH8 && variant != GBS_VARIANT_PLAIN &&
      variant != GBS_VARIANT_TILE3D && !march3d && P->prob.op != GBS_ACOUSTIC2D)
    return fail(GBS_EUNSUPPORTED, "this variant is not built for this operator");
  P->variant = variant;
  return GBS_OK;
}

extern "C" int gbs_plan_set_band(gbs_plan* P, int32_t rows) {
  if (!P) return fail(GBS_EINVAL, "plan is null");
  if (rows < 0 || rows > (1 << 20)) return fail(GBS_EINVAL, "rows per band out of range");
  P->band = rows;
  return GBS_OK;
}

extern "C" int gbs_plan_set_form(gbs_plan* P, int32_t form) {
  if (!P) return fail(GBS_EINVAL, "plan is null");
  if (form & ~(GBS_FORM_SHARED_F0 | GBS_FORM_FUSED_COMBINE | GBS_FORM_ALIGNED_FIRST))
    return fail(GBS_EINVAL, "unknown form flags 0x%x", form);
  P->form = form;
  return GBS_OK;
}

extern "C" int gbs_plan_set_wave_order(gbs_plan* P, int32_t order) {
  if (!P) return fail(GBS_EINVAL, "plan is null");
  if (order < 0 || order > 2) return fail(GBS_EINVAL, "wave order must be 0, 1 or 2");
  P->wave_order = order;
  return GBS_OK;
}

extern "C" int gbs_plan_set_lanes(gbs_plan* P, int32_t lanes) {
  if (!P) return fail(GBS_EINVAL, "plan is null");
  if (lanes < 1 || lanes > GBS_MAX_LANES) return fail(GBS_EINVAL, "lanes must be 1..%d", GBS_MAX_LANES);
  if (lanes > 1 && !P->ev_fork) {
    if (hipEventCreateWithFlags(&P->ev_fork, hipEventDisableTiming) != hipSuccess)
      return fail(GBS_EDEVICE, "creating an event failed");
  }
  for (int l = 1; l < lanes; ++l) {
    if (!P->lane_stream[l] &&
        hipStreamCreateWithFlags(&P->lane_stream[l], hipStreamNonBlocking) != hipSuccess)
      return fail(GBS_EDEVICE, "creating a stream failed");
    if (!P->ev_join[l] &&
        hipEventCreateWithFlags(&P->ev_join[l], hipEventDisableTiming) != hipSuccess)
      return fail(GBS_EDEVICE, "creating an event failed");
  }
  P->lanes = lanes;
  return GBS_OK;
}

namespace {

// Rebind a plan to another caller stream: work enqueued from now on goes to
// `to`, which first waits for everything already enqueued on `from`.
int rebind_stream(hipStream_t& cur, hipStream_t to) {
  if (to == cur) return GBS_OK;
  hipEvent_t e;
  if (hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess)
    return fail(GBS_EDEVICE, "creating an event failed");
  const bool ok = hipEventRecord(e, cur) == hipSuccess && hipStreamWaitEvent(to, e, 0) == hipSuccess;
  hipEventDestroy(e);
  if (!ok) return fail(GBS_EDEVICE, "ordering the new stream after the old one failed");
  cur = to;
  return GBS_OK;
}

}  // namespace

extern "C" int gbs_plan_set_stream(gbs_plan* P, void* hip_stream) {
  if (!P) return fail(GBS_EINVAL, "plan is null");
  return rebind_stream(P->stream, (hipStream_t)hip_stream);
}

extern "C" int gbs_plan_get_variant(const gbs_plan* P, int32_t* variant) {
  if (!P || !variant) return fail(GBS_EINVAL, "null argument");
  *variant = resolve_variant(P);
  return GBS_OK;
}

extern "C" int gbs_plan_autotune(gbs_plan* P, const void* y_in, void* y_out, int32_t macro_steps,
                                 int32_t* variant_out, int32_t* band_out, int32_t* lanes_io) {
  if (!P || !y_in || !y_out || macro_steps < 1) return fail(GBS_EINVAL, "bad arguments");
  if (P->prob.op != GBS_ACOUSTIC2D) {
    // one kernel form for the other operators
    if (variant_out) *variant_out = resolve_variant(P);
    if (band_out) *band_out = P->band;
    if (lanes_io) *lanes_io = P->lanes;
    return GBS_OK;
  }
  const int variants[] = {GBS_VARIANT_TEMPORAL, GBS_VARIANT_TEMPORAL4, GBS_VARIANT_TEMPORAL_S5,
                          GBS_VARIANT_TEMPORAL_S6, GBS_VARIANT_TEMPORAL_WG4,
                          GBS_VARIANT_TEMPORAL_WG8};
  const int bands[] = {0, 32, 64, 96, 128};
  const int fixed = lanes_io ? *lanes_io : 0;
  if (fixed < 0 || fixed > GBS_MAX_LANES) return fail(GBS_EINVAL, "lanes must be 0..%d", GBS_MAX_LANES);
  std::vector<int> lane_counts = {1, 2, 3};
  if (fixed > 0) lane_counts = {fixed};
  hipEvent_t a, b;
  if (hipEventCreate(&a) != hipSuccess || hipEventCreate(&b) != hipSuccess)
    return fail(GBS_EDEVICE, "creating events failed");
  float best = 1e30f;
  int bv = P->variant, bb = P->band, bl = P->lanes;
  int st = GBS_OK;
  for (int lanes : lane_counts) {
    st = gbs_plan_set_lanes(P, lanes);
    if (st) break;
    for (int v : variants) {
      if (P->prob.fd_order == 8 && (v == GBS_VARIANT_TEMPORAL4 || v == GBS_VARIANT_TEMPORAL_S5 ||
                                    v == GBS_VARIANT_TEMPORAL_S6))
        continue;
      for (int band : bands) {
        P->variant = v;
        P->band = band;
        st = gbs_step(P, 0.0, 1, y_in, y_out);              // warm-up
        if (st) break;
        hipEventRecord(a, P->stream);
        st = gbs_step(P, 0.0, macro_steps, y_in, y_out);
        hipEventRecord(b, P->stream);
        if (st) break;
        if (hipEventSynchronize(b) != hipSuccess) {
          st = fail(GBS_EDEVICE, "event sync failed");
          break;
        }
        float ms = 0;
        hipEventElapsedTime(&ms, a, b);
        if (ms < best) { best = ms; bv = v; bb = band; bl = lanes; }
      }
      if (st) break;
    }
    if (st) break;
  }
  hipEventDestroy(a);
  hipEventDestroy(b);
  P->variant = bv;
  P->band = bb;
  if (gbs_plan_set_lanes(P, bl) != GBS_OK && !st) st = GBS_EDEVICE;
  if (st) return st;
  if (variant_out) *variant_out = bv;
  if (band_out) *band_out = bb;
  if (lanes_io) *lanes_io = bl;
  return GBS_OK;
}

extern "C" int gbs_plan_set_timing(gbs_plan* P, int32_t enabled) {
  if (!P) return fail(GBS_EINVAL, "plan is null");
  if (enabled < 0) return fail(GBS_EINVAL, "enabled must be >= 0");
  P->timing = enabled != 0;
  P->lf_used = P->first_used = P->adj_used = 0;
  P->adj_bytes = 0;
  // create the events for `enabled` macro steps up front, so that timed runs
  // do not create events between launches
  if (enabled > 1) {
    size_t lf = (size_t)enabled * P->nmax, fi = (size_t)enabled;
    while (P->lf_ev.size() < lf) next_event(P->lf_ev, P->lf_used);
    while (P->first_ev.size() < fi) next_event(P->first_ev, P->first_used);
    P->lf_used = P->first_used = 0;
  }
  return GBS_OK;
}

extern "C" int gbs_plan_get_adjoint_timing(gbs_plan* P, double* pass_ms, int64_t* pass_n,
                                           double* pass_bytes) {
  if (!P) return fail(GBS_EINVAL, "plan is null");
  if (hipStreamSynchronize(P->stream) != hipSuccess) return fail(GBS_EDEVICE, "stream sync failed");
  double tot = 0;
  for (size_t i = 0; i < P->adj_used; ++i) {
    float ms = 0;
    if (hipEventElapsedTime(&ms, P->adj_ev[i].a, P->adj_ev[i].b) == hipSuccess) tot += ms;
  }
  if (pass_ms) *pass_ms = tot;
  if (pass_n) *pass_n = (int64_t)P->adj_used;
  if (pass_bytes) *pass_bytes = P->adj_bytes;
  P->adj_used = 0;
  P->adj_bytes = 0;
  return GBS_OK;
}

extern "C" int gbs_plan_get_timing(gbs_plan* P, double* lf_ms, int64_t* lf_n, double* first_ms,
                                   int64_t* first_n) {
  if (!P) return fail(GBS_EINVAL, "plan is null");
  if (hipStreamSynchronize(P->stream) != hipSuccess) return fail(GBS_EDEVICE, "stream sync failed");
  auto sum = [](std::vector<EventPair>& pool, size_t used) {
    double tot = 0;
    for (size_t i = 0; i < used; ++i) {
      float ms = 0;
      if (hipEventElapsedTime(&ms, pool[i].a, pool[i].b) == hipSuccess) tot += ms;
    }
    return tot;
  };
  if (lf_ms) *lf_ms = sum(P->lf_ev, P->lf_used);
  if (lf_n) *lf_n = (int64_t)P->lf_used;
  if (first_ms) *first_ms = sum(P->first_ev, P->first_used);
  if (first_n) *first_n = (int64_t)P->first_used;
  P->lf_used = P->first_used = 0;
  return GBS_OK;
}

// Algorithmic HBM bytes of one macro step, per kernel class, for the variant
// in use: every state a launch reads is counted once per launch (y0, which
// the first passes of all sequences share, and the c^2 field, which every
// sequence and right-hand side shares), every level, y* or accumulator it
// writes once; halo re-reads and redundant edge work are not counted.
extern "C" int gbs_plan_algorithmic_bytes(const gbs_plan* P, double* step_bytes,
                                          int64_t* step_launches, double* aux_bytes,
                                          int64_t* aux_launches) {
  if (!P) return fail(GBS_EINVAL, "plan is null");
  const double pts = (double)P->field * P->prob.n_rhs;
  const double Fb = (double)P->F * dsize(P->prob.dtype);   // one level, per point
  const double F8 = (double)P->F * 8.0;                     // one FP64 state, per point
  // the coefficient field, read once per launch (shared by the right-hand sides)
  const double c2b = P->prob.c2_field ? (double)P->field * dsize(P->prob.dtype) : 0.0;
  const int v = resolve_variant(P);
  double sb = 0, ab = 0;
  int64_t sl = 0, al = 0;
  if (P->prob.op == GBS_ACOUSTIC2D && is_temporal(v)) {
    const TemporalShape ts = temporal_shape(v, P->prob.fd_order);
    TemporalForm form;
    const int st = temporal_form(P, ts.G, P->prob.fd_order / 2, ts.wpg, P->prob.fd_order, form);
    if (st) return st;
    const PassSchedule& sch = form.sch;
    const int jl = P->order[P->k - 1];
    for (int j = 0; j < P->k; ++j) {
      const int np = sch.npass[j];
      for (int q = 0; q < np; ++q) {
        if (q > 0) sb += 2 * Fb * pts;                       // the pair of levels in
        if (q < np - 1) sb += 2 * Fb * pts;                  // the pair out
        else if (form.fuse && j == jl) sb += ((P->k - 1) * F8 + Fb) * pts;  // other y*, y_out
        else sb += F8 * pts;                                 // y*
      }
    }
    sl = sch.nrounds;
    // round 0 reads y0 (and F_0) once; c^2 once per launch
    sb += (form.shared_f0 ? 2 : 1) * Fb * pts + sl * c2b;
    if (form.shared_f0) {
      ab += 2 * Fb * pts + c2b;                              // f(t0, y0): y0 in, F_0 out
      al += 1;
    }
    if (!form.fuse) {
      ab += ((double)P->k * F8 + Fb) * pts;                  // combine
      al += 1;
    }
  } else {
    for (int r = 0; r < P->k; ++r) {
      const int N = P->steps[P->order[r]];
      sb += (N - 1) * 3 * Fb * pts;
      double last = 2 * Fb;
      if (r == 0) last += F8;
      else if (r == P->k - 1) last += F8 + Fb;
      else last += 2 * F8;
      sb += last * pts;
    }
    sl = P->nmax;
    sb += sl * c2b;
    ab = (1 + P->k) * Fb * pts + c2b;                        // first evaluation
    al = 1;
  }
  if (step_bytes) *step_bytes = sb;
  if (step_launches) *step_launches = sl;
  if (aux_bytes) *aux_bytes = ab;
  if (aux_launches) *aux_launches = al;
  return GBS_OK;
}

extern "C" int gbs_plan_updates_per_macro_step(const gbs_plan* P, double* updates) {
  if (!P || !updates) return fail(GBS_EINVAL, "null argument");
  int evals = 1;
  for (int j = 0; j < P->k; ++j) evals += P->steps[j];
  *updates = (double)P->field * P->prob.n_rhs * evals;
  return GBS_OK;
}

namespace {

// Releases what a plan created besides itself (lane streams, events).
void plan_release(gbs_plan* P) {
  for (int l = 1; l < GBS_MAX_LANES; ++l) {
    if (P->lane_stream[l]) {
      hipStreamSynchronize(P->lane_stream[l]);
      hipStreamDestroy(P->lane_stream[l]);
    }
    if (P->ev_join[l]) hipEventDestroy(P->ev_join[l]);
  }
  if (P->ev_fork) hipEventDestroy(P->ev_fork);
  for (auto& e : P->lf_ev) { hipEventDestroy(e.a); hipEventDestroy(e.b); }
  for (auto& e : P->first_ev) { hipEventDestroy(e.a); hipEventDestroy(e.b); }
  for (auto& e : P->adj_ev) { hipEventDestroy(e.a); hipEventDestroy(e.b); }
}

}  // namespace

extern "C" int gbs_plan_destroy(gbs_plan* P) {
  if (!P) return GBS_OK;
  plan_release(P);
  delete P;
  return GBS_OK;
}

// ---------------------------------------------------------------------------
// Macro steps without any device allocation (gbs_step_scratch): the plan
// lives on the host stack and its workspace is `scratch`, a static device
// array of the library (one copy per GPU, held until the process ends).  In
// host code `scratch` names a host-side stand-in: its device address comes
// from hipGetSymbolAddress, once per device, and only that address is used.
// ---------------------------------------------------------------------------

static __device__ __align__(256) unsigned char scratch[GBS_SCRATCH_BYTES];

namespace {

constexpr int kScratchDevices = 64;
std::mutex scratch_mu;
void* scratch_dev[kScratchDevices] = {};

// The current device's address of `scratch`.
int scratch_address(void** out) {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return fail(GBS_EDEVICE, "hipGetDevice failed");
  if (dev < 0 || dev >= kScratchDevices) return fail(GBS_EDEVICE, "device %d out of range", dev);
  std::lock_guard<std::mutex> lk(scratch_mu);
  if (!scratch_dev[dev]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p)
      return fail(GBS_EDEVICE, "hipGetSymbolAddress(scratch) failed: %s", hipGetErrorString(e));
    scratch_dev[dev] = p;
  }
  *out = scratch_dev[dev];
  return GBS_OK;
}

}  // namespace

extern "C" int gbs_step_scratch(const gbs_problem* prob, const gbs_scheme* sch, double H,
                                double t0, int32_t n_macro, const void* y_in, void* y_out,
                                void* hip_stream) {
  if (prob && prob->fd_order == GBS_FD_SPECTRAL)
    return fail(GBS_EUNSUPPORTED, "gbs_step_scratch: the Fourier derivative is not offered");
  size_t need = 0;
  int st = gbs_plan_workspace_bytes(prob, sch, &need);
  if (st) return st;
  if (need > GBS_SCRATCH_BYTES)
    return fail(GBS_ENOMEM,
                "gbs_step_scratch: the problem needs %zu bytes of workspace, the static scratch "
                "array holds %zu (use gbs_plan_create with a workspace of your own)",
                need, (size_t)GBS_SCRATCH_BYTES);
  void* ws = nullptr;
  st = scratch_address(&ws);
  if (st) return st;
  gbs_plan P;
  st = plan_init(&P, prob, sch, H, ws, GBS_SCRATCH_BYTES, hip_stream);
  if (!st) st = gbs_step(&P, t0, n_macro, y_in, y_out);
  plan_release(&P);
  return st;
}

extern "C" const char* gbs_last_error(void) { return g_last_error.c_str(); }

// ---------------------------------------------------------------------------
// Batches: many independent 2-D acoustic instances (own grid size, c^2 and H)
// advanced together.  Every pass round of every (instance, sequence) pair is
// one launch over a device-side item table; the combination of all
// instances is one more launch.  A macro step can be captured once in a
// hipGraph and replayed.
// ---------------------------------------------------------------------------

struct gbs_batch_plan {
  int n = 0, k = 0, dtype = GBS_F64, fd_order = 4;
  std::vector<gbs_problem> prob;
  std::vector<double> H;
  int32_t steps[GBS_MAX_SEQ];
  double w[GBS_MAX_SEQ];
  int order[GBS_MAX_SEQ];
  int variant = GBS_VARIANT_TEMPORAL;
  int band = 64;
  hipStream_t stream = nullptr;   // caller's stream
  hipStream_t gstream = nullptr;  // own stream for graph capture and replay
  char* ws = nullptr;
  size_t ws_bytes = 0;
  // device tables (in the workspace) and their host images
  char* tab_dev = nullptr;
  size_t tab_bytes = 0;
  std::vector<char> tab_host;
  std::vector<size_t> round_off;   // byte offset of each round's item table
  std::vector<int> round_items, round_waves;
  size_t comb_off = 0;
  int comb_blocks = 0;
  std::vector<void*> ycache;       // state pointers the tables were built for
  std::vector<std::vector<std::array<std::array<void*, 2>, 2>>> pair;  // [inst][seq][pair][level]
  bool use_graph = false;
  hipGraphExec_t graph = nullptr;
  hipEvent_t ev_in = nullptr, ev_out = nullptr;
};

namespace {

int batch_gmax(int variant, int fd_order) { return temporal_shape(variant, fd_order).G; }

size_t batch_level_bytes(const gbs_problem& p) {
  return align_up((size_t)3 * p.n[0] * p.n[1] * dsize(p.dtype));
}

// upper bound of the item tables: every (instance, sequence) pair in every
// round (at most N_max + 1 rounds) plus one combine item per instance
size_t batch_table_bytes(int n, int k, int nmax) {
  const size_t item = std::max(sizeof(PassItem<double>), sizeof(PassItem<float>));
  const size_t comb = std::max(sizeof(CombineItem<double>), sizeof(CombineItem<float>));
  return align_up((size_t)(nmax + 1) * n * k * item) + (size_t)(nmax + 1) * kAlign +
         align_up((size_t)n * comb);
}

template <typename T>
void batch_build_tables(gbs_batch_plan* B, void* const* y) {
  const int G = batch_gmax(B->variant, B->fd_order);
  const int R = B->fd_order / 2;
  const int wpg = temporal_shape(B->variant, B->fd_order).wpg;
  PassSchedule sch;
  make_schedule(B->steps, B->k, G, R, wpg, sch);
  const int* npass = sch.npass;
  const int maxpass = sch.nrounds;
  B->tab_host.assign(B->tab_bytes, 0);
  B->round_off.assign(maxpass, 0);
  B->round_items.assign(maxpass, 0);
  B->round_waves.assign(maxpass, 0);
  size_t off = 0;
  for (int q = 0; q < maxpass; ++q) {
    B->round_off[q] = off;
    PassItem<T>* items = (PassItem<T>*)(B->tab_host.data() + off);
    int m = 0, waves = 0;
    for (int i = 0; i < B->n; ++i) {
      const gbs_problem& p = B->prob[i];
      const int nx = (int)p.n[0], ny = (int)p.n[1];
      for (int r = 0; r < B->k; ++r) {
        const int j = B->order[r];
        const int rq = q;                               // round
        const int qp = rq - sch.round0[j];              // this sequence's pass in the round
        if (qp < 0 || qp >= npass[j]) continue;
        PassItem<T>& it = items[m++];
        auto& pr = B->pair[i][j];
        it.cur = qp == 0 ? (const T*)y[i] : (const T*)pr[(qp - 1) % 2][1];
        it.old = qp == 0 ? nullptr : (const T*)pr[(qp - 1) % 2][0];
        it.out_a = (T*)pr[qp % 2][0];
        it.out_b = (T*)pr[qp % 2][1];
        it.ystar = (double*)pr[qp % 2][0];
        it.c2f = (const T*)p.c2_field;
        it.field = (int64_t)nx * ny;
        it.h = (T)(B->H[i] / B->steps[j]);
        it.c2c = (T)p.c2;
        const double den = B->fd_order == 8 ? 840.0 : 12.0;
        it.invx = (T)((double)nx / den);
        it.invy = (T)((double)ny / den);
        it.nx = nx;
        it.ny = ny;
        it.g = sch.gsz[j][qp];
        it.flags = (qp == 0 ? PASS_FIRST : 0) | (qp == npass[j] - 1 ? PASS_FINAL : 0);
        const int wv = 64 * temporal_shape(B->variant, B->fd_order).wpg - 2 * it.g * R;
        it.strips = (nx + wv - 1) / wv;
        it.nbands = (ny + B->band - 1) / B->band;
        it.band = B->band;
        it.wave_begin = waves;
        waves += it.strips * it.nbands;
      }
    }
    B->round_items[q] = m;
    B->round_waves[q] = waves;
    off += align_up((size_t)m * sizeof(PassItem<T>));
  }
  B->comb_off = off;
  CombineItem<T>* ci = (CombineItem<T>*)(B->tab_host.data() + off);
  int blocks = 0;
  for (int i = 0; i < B->n; ++i) {
    const gbs_problem& p = B->prob[i];
    CombineItem<T>& c = ci[i];
    c.k = B->k;
    c.n = (int64_t)3 * p.n[0] * p.n[1];
    c.yout = (T*)y[i];
    for (int r = 0; r < B->k; ++r) {
      const int j = B->order[r];
      c.c[r] = B->w[j];
      c.ystar[r] = (const double*)B->pair[i][j][(npass[j] - 1) % 2][0];
    }
    c.block_begin = blocks;
    blocks += (int)((c.n + 255) / 256);
  }
  B->comb_blocks = blocks;
}

template <typename T>
void batch_launch_macro_step(gbs_batch_plan* B, hipStream_t s) {
  const int G = batch_gmax(B->variant, B->fd_order);
  for (size_t q = 0; q < B->round_off.size(); ++q) {
    BatchPassArgs<T> a;
    a.items = (const PassItem<T>*)(B->tab_dev + B->round_off[q]);
    a.n_items = B->round_items[q];
    a.total_waves = B->round_waves[q];
    const int wpg = temporal_shape(B->variant, B->fd_order).wpg;
    const dim3 grid((unsigned)(wpg > 1 ? a.total_waves : (a.total_waves + 3) / 4));
    const dim3 blk(wpg > 1 ? 64 * wpg : 256);
    if (B->fd_order == 8) {
      if (wpg == 4) hipLaunchKernelGGL((pass2d_batch<T, 8, 3, true, 4>), grid, blk, 0, s, a);
      else if (wpg == 8) hipLaunchKernelGGL((pass2d_batch<T, 8, 3, true, 8>), grid, blk, 0, s, a);
      else hipLaunchKernelGGL((pass2d_batch<T, 8, 3, true, 1>), grid, blk, 0, s, a);
    } else if (wpg == 4) {
      hipLaunchKernelGGL((pass2d_batch<T, 4, 7, false, 4>), grid, blk, 0, s, a);
    } else if (wpg == 8) {
      hipLaunchKernelGGL((pass2d_batch<T, 4, 7, false, 8>), grid, blk, 0, s, a);
    } else if (G == 4) {
      hipLaunchKernelGGL((pass2d_batch<T, 4, 4, false, 1>), grid, blk, 0, s, a);
    } else if (G == 5) {
      hipLaunchKernelGGL((pass2d_batch<T, 4, 5, true, 1>), grid, blk, 0, s, a);
    } else if (G == 6) {
      hipLaunchKernelGGL((pass2d_batch<T, 4, 6, true, 1>), grid, blk, 0, s, a);
    } else {
      hipLaunchKernelGGL((pass2d_batch<T, 4, 7, false, 1>), grid, blk, 0, s, a);
    }
  }
  hipLaunchKernelGGL((combine_batch<T>), dim3((unsigned)B->comb_blocks), dim3(256), 0, s,
                     (const CombineItem<T>*)(B->tab_dev + B->comb_off), B->n, B->comb_blocks);
}

void batch_drop_graph(gbs_batch_plan* B) {
  if (B->graph) {
    hipGraphExecDestroy(B->graph);
    B->graph = nullptr;
  }
}

// (Re)build and upload the item tables when the state pointers change.
int batch_prepare(gbs_batch_plan* B, void* const* y) {
  bool same = (int)B->ycache.size() == B->n;
  for (int i = 0; same && i < B->n; ++i) same = B->ycache[i] == y[i];
  if (same && !B->tab_host.empty()) return GBS_OK;
  if (hipStreamSynchronize(B->stream) != hipSuccess) return fail(GBS_EDEVICE, "stream sync failed");
  if (B->gstream && hipStreamSynchronize(B->gstream) != hipSuccess)
    return fail(GBS_EDEVICE, "stream sync failed");
  if (B->dtype == GBS_F64) batch_build_tables<double>(B, y);
  else batch_build_tables<float>(B, y);
  if (hipMemcpy(B->tab_dev, B->tab_host.data(), B->tab_bytes, hipMemcpyHostToDevice) != hipSuccess)
    return fail(GBS_EDEVICE, "uploading the batch tables failed");
  B->ycache.assign(y, y + B->n);
  batch_drop_graph(B);
  return GBS_OK;
}

int batch_run(gbs_batch_plan* B, int n_macro) {
  if (!B->use_graph) {
    for (int m = 0; m < n_macro; ++m) {
      if (B->dtype == GBS_F64) batch_launch_macro_step<double>(B, B->stream);
      else batch_launch_macro_step<float>(B, B->stream);
    }
  } else {
    if (!B->gstream && hipStreamCreateWithFlags(&B->gstream, hipStreamNonBlocking) != hipSuccess)
      return fail(GBS_EDEVICE, "creating the graph stream failed");
    if (!B->ev_in && (hipEventCreateWithFlags(&B->ev_in, hipEventDisableTiming) != hipSuccess ||
                      hipEventCreateWithFlags(&B->ev_out, hipEventDisableTiming) != hipSuccess))
      return fail(GBS_EDEVICE, "creating events failed");
    if (!B->graph) {
      hipGraph_t g = nullptr;
      if (hipStreamBeginCapture(B->gstream, hipStreamCaptureModeThreadLocal) != hipSuccess)
        return fail(GBS_EDEVICE, "graph capture failed to start");
      if (B->dtype == GBS_F64) batch_launch_macro_step<double>(B, B->gstream);
      else batch_launch_macro_step<float>(B, B->gstream);
      if (hipStreamEndCapture(B->gstream, &g) != hipSuccess)
        return fail(GBS_EDEVICE, "graph capture failed");
      const hipError_t e = hipGraphInstantiate(&B->graph, g, nullptr, nullptr, 0);
      hipGraphDestroy(g);
      if (e != hipSuccess) return fail(GBS_EDEVICE, "graph instantiation failed");
    }
    // order the replays after the caller's stream and the caller's stream after them
    hipEventRecord(B->ev_in, B->stream);
    hipStreamWaitEvent(B->gstream, B->ev_in, 0);
    for (int m = 0; m < n_macro; ++m)
      if (hipGraphLaunch(B->graph, B->gstream) != hipSuccess)
        return fail(GBS_EDEVICE, "graph launch failed");
    hipEventRecord(B->ev_out, B->gstream);
    hipStreamWaitEvent(B->stream, B->ev_out, 0);
  }
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return fail(GBS_EDEVICE, "kernel launch failed: %s", hipGetErrorString(e));
  return GBS_OK;
}

int batch_validate(int n_inst, const gbs_problem* probs, const gbs_scheme* sch, const double* H) {
  if (n_inst < 1 || !probs || !H) return fail(GBS_EINVAL, "batch: empty or null arguments");
  int st = validate_scheme(sch);
  if (st) return st;
  for (int i = 0; i < n_inst; ++i) {
    st = validate_problem(&probs[i]);
    if (st) return st;
    if (probs[i].op != GBS_ACOUSTIC2D || probs[i].n_rhs != 1)
      return fail(GBS_EUNSUPPORTED, "batch instance %d: only 2-D acoustic, one right-hand side", i);
    if (probs[i].dtype != probs[0].dtype || probs[i].fd_order != probs[0].fd_order)
      return fail(GBS_EINVAL, "batch instance %d: dtype and stencil order must match", i);
    if (!(H[i] > 0) || !std::isfinite(H[i])) return fail(GBS_EINVAL, "batch instance %d: bad H", i);
    st = check_stable(&probs[i], sch, H[i]);
    if (st) return fail(st, "batch instance %d: %s", i, gbs_last_error());
  }
  return GBS_OK;
}

size_t batch_bytes(int n_inst, const gbs_problem* probs, const gbs_scheme* sch) {
  int nmax = 0;
  for (int j = 0; j < sch->k; ++j) nmax = std::max(nmax, (int)sch->steps[j]);
  size_t b = batch_table_bytes(n_inst, sch->k, nmax);
  for (int i = 0; i < n_inst; ++i) b += 4 * (size_t)sch->k * batch_level_bytes(probs[i]);
  return b;
}

}  // namespace

extern "C" int gbs_batch_workspace_bytes(int32_t n_inst, const gbs_problem* probs,
                                         const gbs_scheme* sch, size_t* bytes) {
  if (!bytes) return fail(GBS_EINVAL, "bytes is null");
  if (n_inst < 1 || !probs) return fail(GBS_EINVAL, "batch: empty or null arguments");
  int st = validate_scheme(sch);
  if (st) return st;
  for (int i = 0; i < n_inst; ++i) {
    st = validate_problem(&probs[i]);
    if (st) return st;
  }
  *bytes = batch_bytes(n_inst, probs, sch);
  return GBS_OK;
}

extern "C" int gbs_batch_plan_create(gbs_batch_plan** out, int32_t n_inst, const gbs_problem* probs,
                                     const gbs_scheme* sch, const double* H, void* workspace,
                                     size_t ws_bytes, void* hip_stream) {
  try {
    if (!out) return fail(GBS_EINVAL, "out is null");
    *out = nullptr;
    int st = batch_validate(n_inst, probs, sch, H);
    if (st) return st;
    if (!workspace || (uintptr_t)workspace % kAlign)
      return fail(GBS_EINVAL, "workspace must be non-null and 256-byte aligned");
    const size_t need = batch_bytes(n_inst, probs, sch);
    if (ws_bytes < need) return fail(GBS_ENOMEM, "workspace has %zu bytes, needs %zu", ws_bytes, need);
    gbs_batch_plan* B = new gbs_batch_plan();
    B->n = n_inst;
    B->k = sch->k;
    B->dtype = probs[0].dtype;
    B->fd_order = probs[0].fd_order;
    B->prob.assign(probs, probs + n_inst);
    B->H.assign(H, H + n_inst);
    int nmax = 0;
    for (int j = 0; j < sch->k; ++j) {
      B->steps[j] = sch->steps[j];
      B->w[j] = sch->weights[j];
      B->order[j] = j;
      nmax = std::max(nmax, (int)sch->steps[j]);
    }
    std::sort(B->order, B->order + B->k, [&](int a, int b) { return B->steps[a] < B->steps[b]; });
    B->stream = (hipStream_t)hip_stream;
    B->ws = (char*)workspace;
    B->ws_bytes = ws_bytes;
    B->tab_dev = B->ws;
    B->tab_bytes = batch_table_bytes(n_inst, sch->k, nmax);
    char* base = B->ws + B->tab_bytes;
    B->pair.resize(n_inst);
    for (int i = 0; i < n_inst; ++i) {
      const size_t lb = batch_level_bytes(probs[i]);
      B->pair[i].resize(sch->k);
      for (int j = 0; j < sch->k; ++j)
        for (int q = 0; q < 2; ++q)
          for (int l = 0; l < 2; ++l) {
            B->pair[i][j][q][l] = base;
            base += lb;
          }
    }
    *out = B;
    return GBS_OK;
  } catch (const std::exception& e) {
    return fail(GBS_EINVAL, "gbs_batch_plan_create: %s", e.what());
  }
}

extern "C" int gbs_batch_set_variant(gbs_batch_plan* B, int32_t variant, int32_t band) {
  if (!B) return fail(GBS_EINVAL, "plan is null");
  if (variant != 0 && !is_temporal(variant))
    return fail(GBS_EUNSUPPORTED, "batches use the temporally blocked variants");
  if (band < 0 || band > (1 << 20)) return fail(GBS_EINVAL, "band out of range");
  if (variant) B->variant = variant;
  if (band) B->band = band;
  B->ycache.clear();       // tables and graph are rebuilt on the next step
  B->tab_host.clear();
  batch_drop_graph(B);
  return GBS_OK;
}

extern "C" int gbs_batch_set_graph(gbs_batch_plan* B, int32_t enabled) {
  if (!B) return fail(GBS_EINVAL, "plan is null");
  B->use_graph = enabled != 0;
  return GBS_OK;
}

extern "C" int gbs_batch_set_stream(gbs_batch_plan* B, void* hip_stream) {
  if (!B) return fail(GBS_EINVAL, "plan is null");
  return rebind_stream(B->stream, (hipStream_t)hip_stream);
}

extern "C" int gbs_batch_step(gbs_batch_plan* B, int32_t n_macro, void* const* y) {
  if (!B || !y) return fail(GBS_EINVAL, "null argument");
  if (n_macro < 0) return fail(GBS_EINVAL, "n_macro must be >= 0");
  for (int i = 0; i < B->n; ++i)
    if (!y[i]) return fail(GBS_EINVAL, "state %d is null", i);
  if (n_macro == 0) return GBS_OK;
  int st = batch_prepare(B, y);
  if (st) return st;
  return batch_run(B, n_macro);
}

extern "C" int gbs_batch_autotune(gbs_batch_plan* B, void* const* y, int32_t macro_steps,
                                  int32_t* variant_out, int32_t* band_out) {
  if (!B || !y || macro_steps < 1) return fail(GBS_EINVAL, "bad arguments");
  const int variants[] = {GBS_VARIANT_TEMPORAL, GBS_VARIANT_TEMPORAL4, GBS_VARIANT_TEMPORAL_S5,
                          GBS_VARIANT_TEMPORAL_S6, GBS_VARIANT_TEMPORAL_WG4,
                          GBS_VARIANT_TEMPORAL_WG8};
  const int bands[] = {32, 64, 96, 128};
  hipEvent_t a, b;
  if (hipEventCreate(&a) != hipSuccess || hipEventCreate(&b) != hipSuccess)
    return fail(GBS_EDEVICE, "creating events failed");
  const bool graph = B->use_graph;
  B->use_graph = false;
  float best = 1e30f;
  int bv = B->variant, bb = B->band;
  for (int v : variants) {
    if (B->fd_order == 8 && (v == GBS_VARIANT_TEMPORAL4 || v == GBS_VARIANT_TEMPORAL_S5 ||
                             v == GBS_VARIANT_TEMPORAL_S6))
      continue;
    for (int band : bands) {
      gbs_batch_set_variant(B, v, band);
      int st = gbs_batch_step(B, 1, y);                  // warm-up (and table upload)
      if (st) { hipEventDestroy(a); hipEventDestroy(b); B->use_graph = graph; return st; }
      hipEventRecord(a, B->stream);
      st = gbs_batch_step(B, macro_steps, y);
      hipEventRecord(b, B->stream);
      if (st || hipEventSynchronize(b) != hipSuccess) {
        hipEventDestroy(a);
        hipEventDestroy(b);
        B->use_graph = graph;
        return st ? st : fail(GBS_EDEVICE, "event sync failed");
      }
      float ms = 0;
      hipEventElapsedTime(&ms, a, b);
      if (ms < best) { best = ms; bv = v; bb = band; }
    }
  }
  hipEventDestroy(a);
  hipEventDestroy(b);
  gbs_batch_set_variant(B, bv, bb);
  B->use_graph = graph;
  if (variant_out) *variant_out = bv;
  if (band_out) *band_out = bb;
  return GBS_OK;
}

extern "C" int gbs_batch_updates_per_macro_step(const gbs_batch_plan* B, double* updates) {
  if (!B || !updates) return fail(GBS_EINVAL, "null argument");
  int evals = 1;
  for (int j = 0; j < B->k; ++j) evals += B->steps[j];
  double pts = 0;
  for (const auto& p : B->prob) pts += (double)p.n[0] * p.n[1];
  *updates = pts * evals;
  return GBS_OK;
}

extern "C" int gbs_batch_plan_destroy(gbs_batch_plan* B) {
  if (!B) return GBS_OK;
  if (B->gstream) hipStreamSynchronize(B->gstream);
  batch_drop_graph(B);
  if (B->gstream) hipStreamDestroy(B->gstream);
  if (B->ev_in) hipEventDestroy(B->ev_in);
  if (B->ev_out) hipEventDestroy(B->ev_out);
  delete B;
  return GBS_OK;
}

// ---------------------------------------------------------------------------
// Receivers, recorded forward runs and the adjoint macro step.
// ---------------------------------------------------------------------------

extern "C" int gbs_plan_set_receivers(gbs_plan* P, int32_t n_rec, const int32_t* rhs,
                                      const int64_t* flat_index) {
  if (!P) return fail(GBS_EINVAL, "plan is null");
  if (n_rec < 0 || n_rec > GBS_MAX_REC) return fail(GBS_EINVAL, "n_rec out of range");
  if (P->prob.op == GBS_ADVECT1D && n_rec) return fail(GBS_EINVAL, "receivers need an acoustic plan");
  if (n_rec && (!rhs || !flat_index)) return fail(GBS_EINVAL, "receiver arrays are null");
  std::vector<RecDesc> r(std::max(n_rec, 1));
  for (int i = 0; i < n_rec; ++i) {
    if (rhs[i] < 0 || rhs[i] >= P->prob.n_rhs || flat_index[i] < 0 || flat_index[i] >= P->field)
      return fail(GBS_EINVAL, "receiver %d out of range", i);
    r[i].idx = flat_index[i];
    r[i].rhs = rhs[i];
    r[i].pad = 0;
  }
  if (n_rec && (hipMemcpyAsync(P->rec_dev, r.data(), n_rec * sizeof(RecDesc),
                               hipMemcpyHostToDevice, P->stream) != hipSuccess ||
                hipStreamSynchronize(P->stream) != hipSuccess))
    return fail(GBS_EDEVICE, "copying the receivers to the workspace failed");
  std::vector<std::pair<int32_t, int64_t>> keys(n_rec);
  for (int i = 0; i < n_rec; ++i) keys[i] = {rhs[i], flat_index[i]};
  std::sort(keys.begin(), keys.end());
  P->rec_distinct = std::adjacent_find(keys.begin(), keys.end()) == keys.end();
  P->nrec = n_rec;
  return GBS_OK;
}

extern "C" int gbs_step_record(gbs_plan* P, double t0, int32_t n_macro, const void* y_in,
                               void* y_out, void* traces) {
  if (!P || !y_in || !y_out || (!traces && P->nrec)) return fail(GBS_EINVAL, "null argument");
  if (n_macro < 0) return fail(GBS_EINVAL, "n_macro must be >= 0");
  const size_t b = dsize(P->prob.dtype);
  for (int m = 0; m < n_macro; ++m) {
    int st = gbs_step(P, t0 + m * P->H, 1, m == 0 ? y_in : y_out, y_out);
    if (st) return st;
    if (P->nrec) {
      const unsigned blocks = (unsigned)((P->nrec + 255) / 256);
      char* out = (char*)traces + (size_t)m * P->nrec * b;
      if (P->prob.dtype == GBS_F64)
        hipLaunchKernelGGL(gather_kernel<double>, dim3(blocks), dim3(256), 0, P->stream,
                           (const double*)y_out, P->state, P->rec_dev, P->nrec, (double*)out);
      else
        hipLaunchKernelGGL(gather_kernel<float>, dim3(blocks), dim3(256), 0, P->stream,
                           (const float*)y_out, P->state, P->rec_dev, P->nrec, (float*)out);
    }
  }
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return fail(GBS_EDEVICE, "kernel launch failed: %s", hipGetErrorString(e));
  return GBS_OK;
}

namespace {

// The temporally blocked adjoint serves the 2-D FD4 operator whenever the
// plan's forward form is a blocked one.
bool blocked_adjoint(const gbs_plan* P) {
  return P->prob.op == GBS_ACOUSTIC2D && P->prob.fd_order == 4 && is_temporal(resolve_variant(P));
}

size_t adjoint_bytes(const gbs_plan* P) {
  const size_t elems = (size_t)P->prob.n_rhs * P->state;
  const size_t lb = align_up(elems * dsize(P->prob.dtype));
  const size_t lbd = align_up(elems * 8);
  const size_t streaming = (size_t)(P->nmax + 2) * lb + 2 * lbd;
  if (P->prob.op != GBS_ACOUSTIC2D || P->prob.fd_order != 4) return streaming;
  // blocked: per sequence two pairs of Z levels (Y and Psi: two states
  // each), lambda_0 + lambda_1 and h lambda_1 (FP64), a gradient field per
  // right-hand side; then the sums over the sequences
  const size_t gb = align_up((size_t)P->prob.n_rhs * P->field * 8);
  const size_t blocked = (size_t)P->k * (8 * lb + 2 * lbd + gb) + 2 * lbd;
  return std::max(streaming, blocked);
}

// G of the blocked adjoint passes (six fields per level in registers).
template <typename T>
constexpr int adj_pass_g() { return sizeof(T) == 8 ? 3 : 4; }

// The forward levels (y_{N-1}, y_N) of every sequence from y_0: blocked
// passes of the plan's forward form (G = 7) over N evaluations, the last
// pass storing its last two levels.  pair_out[j] receives the pair.
template <typename T, int G, bool SKEW1>
int forward_pairs(gbs_plan* P, double t0, const T* y0, const T* pair_out[GBS_MAX_SEQ][2],
                  const int* lane_of, int lane, int lanes, hipStream_t stream) {
  constexpr int ORDER = 4, R = 2;
  PassSchedule sch;
  int st = make_schedule(P->steps, P->k, G, R, 1, sch, false, 0);
  if (st) return st;
  PassArgs<T> pa;
  std::memset(&pa, 0, sizeof(pa));
  T c2c, invz;
  fill_geometry<T>(P, pa.g, c2c, pa.c2f, pa.invx, pa.invy, invz);
  pa.c2c = c2c;
  pa.src_dev = P->src_dev;
  const int nx = (int)P->prob.n[0];
  constexpr int S = SKEW1 ? R + 1 : R;
  const int slots_c = resident_waves(pass2d<T, ORDER, G, SKEW1, 1, false>, 256);
  const int slots_v = resident_waves(pass2d<T, ORDER, G, SKEW1, 1, true>, 256);
  const int slots = std::max(1, (P->prob.c2_field ? slots_v : slots_c) / lanes);
  for (int rr = 0; rr < sch.nrounds; ++rr) {
    int n = 0, maxs = 0;
    for (int r = 0; r < P->k; ++r) {
      const int j = P->order[r];
      const int q = rr - sch.round0[j];
      if (lane_of[r] != lane || q < 0 || q >= sch.npass[j]) continue;
      PassSeq<T>& d = pa.seq[n++];
      const double h = P->H / P->steps[j];
      int s0 = 0;
      for (int qq = 0; qq < q; ++qq) s0 += sch.gsz[j][qq];
      d.g = sch.gsz[j][q];
      d.h = (T)h;
      d.flags = q == 0 ? PASS_FIRST : 0;
      d.cur = q == 0 ? y0 : (const T*)P->pair[j][(q - 1) % 2][1];
      d.old = q == 0 ? nullptr : (const T*)P->pair[j][(q - 1) % 2][0];
      d.out_a = (T*)P->pair[j][q % 2][0];
      d.out_b = (T*)P->pair[j][q % 2][1];
      d.ystar = nullptr;
      d.strips = (nx + (64 - 2 * d.g * R) - 1) / (64 - 2 * d.g * R);
      for (int e = 0; e < d.g; ++e)
        d.amp[e] = P->nsrc ? ricker(t0 + (s0 + e) * h, P->f0, P->delay) : 0.0;
      maxs = std::max(maxs, d.strips);
    }
    if (n == 0) continue;
    pa.max_strips = maxs;
    {
      int strips = 0, gmax = 0;
      for (int i = 0; i < n; ++i) {
        strips += pa.seq[i].strips;
        gmax = std::max(gmax, pa.seq[i].g);
      }
      pa.band = band_for_round(P, strips, gmax, R, S, slots);
      pa.nbands = (int)((P->prob.n[1] + pa.band - 1) / pa.band);
    }
    const unsigned blocks = ((unsigned)maxs * pa.nbands + 3) / 4;
    const dim3 grid(blocks, n, P->prob.n_rhs), blk(256);
    if (P->prob.c2_field)
      hipLaunchKernelGGL((pass2d<T, ORDER, G, SKEW1, 1, true>), grid, blk, 0, stream, pa);
    else
      hipLaunchKernelGGL((pass2d<T, ORDER, G, SKEW1, 1, false>), grid, blk, 0, stream, pa);
  }
  for (int j = 0; j < P->k; ++j) {
    const int q = sch.npass[j] - 1;
    pair_out[j][0] = (const T*)P->pair[j][q % 2][0];   // y_{N-1}
    pair_out[j][1] = (const T*)P->pair[j][q % 2][1];   // y_N
  }
  return GBS_OK;
}

// Sums over the sequences (ascending N) of the blocked adjoint's outputs.
template <typename T>
struct AdjSumArgs {
  const double* ysum[GBS_MAX_SEQ];
  const double* f1[GBS_MAX_SEQ];
  const double* gsum[GBS_MAX_SEQ];
  double* yacc;
  double* facc;
  double* grad;        // or null
  int64_t n;           // elements of one whole state
  int64_t field;
  int32_t k, nrhs;
};

// The sums run in ascending sequence order (and right-hand side order for
// the gradient); the loads of up to 8 terms are issued before they are
// added, since a loop over the runtime count alone waits for each load.
template <typename T>
__global__ __launch_bounds__(256) void adj_sum_kernel(const AdjSumArgs<T> a) {
  constexpr int CH = 8;
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= a.n) return;
  double ys = 0.0, fs = 0.0;
  for (int r0 = 0; r0 < a.k; r0 += CH) {
    double y[CH], f[CH];
#pragma unroll
    for (int u = 0; u < CH; ++u) {
      y[u] = r0 + u < a.k ? a.ysum[r0 + u][i] : 0.0;
      f[u] = r0 + u < a.k ? a.f1[r0 + u][i] : 0.0;
    }
#pragma unroll
    for (int u = 0; u < CH; ++u) {
      if (r0 + u < a.k) {
        ys = r0 + u == 0 ? y[u] : ys + y[u];
        fs = r0 + u == 0 ? f[u] : fs + f[u];
      }
    }
  }
  a.yacc[i] = ys;
  a.facc[i] = fs;
  if (a.grad && i < a.field) {
    // terms t = r nrhs + q: sequence r, right-hand side q
    const int nt = a.k * a.nrhs;
    double gs = 0.0;
    for (int t0 = 0; t0 < nt; t0 += CH) {
      double g[CH];
#pragma unroll
      for (int u = 0; u < CH; ++u) {
        const int t = t0 + u;
        g[u] = t < nt ? a.gsum[t / a.nrhs][(int64_t)(t % a.nrhs) * a.field + i] : 0.0;
      }
#pragma unroll
      for (int u = 0; u < CH; ++u)
        if (t0 + u < nt) gs += g[u];
    }
    a.grad[i] += gs;
  }
}

// Algorithmic HBM bytes of one blocked adjoint pass launch over its n
// sequences: a first pass reads y_N, y_{N-1} and ybar, a later one the two Z
// levels (Y and Psi, four states); a pass writes two Z levels, or (final)
// lambda_0 + lambda_1 and h lambda_1 in FP64; the gradient row sums are
// written (first pass) or read and written (later) once per point and
// right-hand side; c^2 is read once per launch.
template <typename T>
double adj_launch_bytes(const gbs_plan* P, const AdjPassArgs<T>& pa, int n, size_t b) {
  const double pts = (double)P->field * P->prob.n_rhs;
  const double Fb = 3.0 * b, F8 = 3.0 * 8;
  double tot = P->prob.c2_field ? (double)P->field * b : 0.0;
  for (int i = 0; i < n; ++i) {
    const AdjPassSeq<T>& d = pa.seq[i];
    const bool first = d.flags & ADJ_FIRST, final_ = d.flags & ADJ_FINAL;
    tot += ((first ? 3 * Fb : 4 * Fb) + (final_ ? 2 * F8 : 4 * Fb) + (first ? 8.0 : 16.0)) * pts;
  }
  return tot;
}

template <typename T>
int adjoint_blocked_run(gbs_plan* P, double t0, const T* y0, T* ybar, const T* tbar,
                        double* grad, char* ws, const T* kept = nullptr) {
  constexpr int ORDER = 4, R = 2;
  constexpr int G = adj_pass_g<T>();
  const size_t elems = (size_t)P->prob.n_rhs * P->state;
  const size_t lb = align_up(elems * sizeof(T));
  const size_t lbd = align_up(elems * 8);
  const size_t gb = align_up((size_t)P->prob.n_rhs * P->field * 8);
  hipStream_t s = P->stream;
  // workspace: per sequence [Z pairs: 8 lb][ysum][f1][gsum], then yacc, facc
  struct SeqBufs { T* z[2][2]; double* ysum; double* f1; double* gsum; } bufs[GBS_MAX_SEQ];
  char* cur = ws;
  for (int j = 0; j < P->k; ++j) {
    for (int q = 0; q < 2; ++q)
      for (int l = 0; l < 2; ++l) { bufs[j].z[q][l] = (T*)cur; cur += 2 * lb; }
    bufs[j].ysum = (double*)cur; cur += lbd;
    bufs[j].f1 = (double*)cur; cur += lbd;
    bufs[j].gsum = (double*)cur; cur += gb;
  }
  double* yacc = (double*)cur; cur += lbd;
  double* facc = (double*)cur;

  if (tbar && P->nrec)
    hipLaunchKernelGGL(inject_kernel<T>, dim3((unsigned)((P->nrec + 255) / 256)), dim3(256), 0, s,
                       ybar, P->state, P->rec_dev, P->nrec, tbar, (int)P->rec_distinct);
  // lanes as for the forward passes: folded pairs of sequences, each lane's
  // forward pairs and backward passes on its own stream
  const int L = std::max(1, std::min(P->lanes, P->k));
  int lane_of[GBS_MAX_SEQ];
  for (int r = 0; r < P->k; ++r) lane_of[r] = std::min(r, P->k - 1 - r) % L;
  if (L > 1) {
    hipEventRecord(P->ev_fork, s);
    for (int l = 1; l < L; ++l) hipStreamWaitEvent(P->lane_stream[l], P->ev_fork, 0);
  }
  PassSchedule sch;
  int st = make_schedule(P->steps, P->k, G, R, 1, sch, false, 0);
  if (st) return st;
  const T* pairs[GBS_MAX_SEQ][2];
  if (kept) {
    // (y_{N-1}, y_N) kept by gbs_step_keep_pairs: [sequence j][2][whole state]
    for (int j = 0; j < P->k; ++j) {
      pairs[j][0] = kept + (size_t)(2 * j) * elems;
      pairs[j][1] = kept + (size_t)(2 * j + 1) * elems;
    }
  }
  for (int l = 0; l < L; ++l) {
    const hipStream_t ls = l == 0 ? s : P->lane_stream[l];
    // the forward pairs with the pass shape of the plan's forward form
    // (its evaluations per pass and time skew; one wavefront per strip)
    if (!kept) {
      switch (temporal_shape(resolve_variant(P), 4).G) {
        case 4: st = forward_pairs<T, 4, false>(P, t0, y0, pairs, lane_of, l, L, ls); break;
        case 5: st = forward_pairs<T, 5, true>(P, t0, y0, pairs, lane_of, l, L, ls); break;
        case 6: st = forward_pairs<T, 6, true>(P, t0, y0, pairs, lane_of, l, L, ls); break;
        default: st = forward_pairs<T, 7, false>(P, t0, y0, pairs, lane_of, l, L, ls); break;
      }
    }
    if (st) return st;
    AdjPassArgs<T> pa;
    std::memset(&pa, 0, sizeof(pa));
    T c2c, invz;
    fill_geometry<T>(P, pa.g, c2c, pa.c2f, pa.invx, pa.invy, invz);
    pa.c2c = c2c;
    pa.src_dev = P->src_dev;
    pa.zstride = (int64_t)elems;
    const int nx = (int)P->prob.n[0];
    const int slots_c = resident_waves(adj_pass2d<T, G, false>, 256);
    const int slots_v = resident_waves(adj_pass2d<T, G, true>, 256);
    const int slots = std::max(1, (P->prob.c2_field ? slots_v : slots_c) / L);
    for (int rr = 0; rr < sch.nrounds; ++rr) {
      int n = 0, maxs = 0;
      for (int r = 0; r < P->k; ++r) {
        const int j = P->order[r];
        const int q = rr - sch.round0[j];
        if (lane_of[r] != l || q < 0 || q >= sch.npass[j]) continue;
        AdjPassSeq<T>& d = pa.seq[n++];
        const int N = P->steps[j];
        const double h = P->H / N;
        // the pass's input level is Z_{s0}: s0 = -1 for the first pass
        int s0 = -1;
        for (int qq = 0; qq < q; ++qq) s0 += sch.gsz[j][qq];
        d.g = sch.gsz[j][q];
        d.h = (T)h;
        d.half_cw = (T)(0.5 * P->w[j]);
        d.flags = (q == 0 ? ADJ_FIRST : 0) | (q == sch.npass[j] - 1 ? ADJ_FINAL : 0);
        d.cur = q == 0 ? pairs[j][1] : bufs[j].z[(q - 1) % 2][1];
        d.old = q == 0 ? pairs[j][0] : bufs[j].z[(q - 1) % 2][0];
        d.ybar = ybar;
        d.out_a = bufs[j].z[q % 2][0];
        d.out_b = bufs[j].z[q % 2][1];
        d.ysum = bufs[j].ysum;
        d.f1 = bufs[j].f1;
        d.gsum = bufs[j].gsum;
        d.strips = (nx + (64 - 2 * d.g * R) - 1) / (64 - 2 * d.g * R);
        // evaluation e+1 applies f to Y of level e, y_{N - s0 - e - 1}
        for (int e = 0; e < d.g; ++e)
          d.amp[e] = P->nsrc ? ricker(t0 + (N - s0 - e - 1) * h, P->f0, P->delay) : 0.0;
        maxs = std::max(maxs, d.strips);
      }
      if (n == 0) continue;
      pa.max_strips = maxs;
      {
        int strips = 0, gmax = 0;
        for (int q2 = 0; q2 < n; ++q2) {
          strips += pa.seq[q2].strips;
          gmax = std::max(gmax, pa.seq[q2].g);
        }
        pa.band = band_for_round(P, strips, gmax, R, R, slots);
        pa.nbands = (int)((P->prob.n[1] + pa.band - 1) / pa.band);
      }
      const unsigned blocks = ((unsigned)maxs * pa.nbands + 3) / 4;
      const dim3 grid(blocks, n, P->prob.n_rhs), blk(256);
      EventPair* ev = nullptr;
      if (P->timing && L == 1) {
        ev = &next_event(P->adj_ev, P->adj_used);
        hipEventRecord(ev->a, ls);
        P->adj_bytes += adj_launch_bytes(P, pa, n, sizeof(T));
      }
      if (P->prob.c2_field)
        hipLaunchKernelGGL((adj_pass2d<T, G, true>), grid, blk, 0, ls, pa);
      else
        hipLaunchKernelGGL((adj_pass2d<T, G, false>), grid, blk, 0, ls, pa);
      if (ev) hipEventRecord(ev->b, ls);
    }
  }  // lanes
  if (L > 1) {
    for (int l = 1; l < L; ++l) {
      hipEventRecord(P->ev_join[l], P->lane_stream[l]);
      hipStreamWaitEvent(s, P->ev_join[l], 0);
    }
  }
  AdjSumArgs<T> sa;
  std::memset(&sa, 0, sizeof(sa));
  for (int r = 0; r < P->k; ++r) {
    const int j = P->order[r];
    sa.ysum[r] = bufs[j].ysum;
    sa.f1[r] = bufs[j].f1;
    sa.gsum[r] = bufs[j].gsum;
  }
  sa.yacc = yacc;
  sa.facc = facc;
  sa.grad = grad;
  sa.n = (int64_t)elems;
  sa.field = P->field;
  sa.k = P->k;
  sa.nrhs = P->prob.n_rhs;
  hipLaunchKernelGGL((adj_sum_kernel<T>), dim3((unsigned)((elems + 255) / 256)), dim3(256), 0, s,
                     sa);
  AdjFinalArgs<T> fz;
  std::memset(&fz, 0, sizeof(fz));
  T ix, iy, iz;
  fill_geometry<T>(P, fz.g, fz.c2c, fz.c2f, ix, iy, iz);
  fz.invx = (double)P->prob.n[0] / 12.0;
  fz.invy = (double)P->prob.n[1] / 12.0;
  fz.invz = (double)P->prob.n[2] / 12.0;
  fz.yacc = yacc;
  fz.facc = facc;
  fz.y0 = y0;
  fz.ybar = ybar;
  fz.grad = grad;
  fz.nrhs = P->prob.n_rhs;
  const unsigned gx = (unsigned)((P->field + 255) / 256);
  hipLaunchKernelGGL((adj_final_kernel<T, ORDER, OP_AC2D>), dim3(gx), dim3(256), 0, s, fz);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return fail(GBS_EDEVICE, "kernel launch failed: %s", hipGetErrorString(e));
  return GBS_OK;
}

template <typename T, int ORDER, int OP>
int adjoint_run(gbs_plan* P, double t0, const T* y0, T* ybar, const T* tbar, double* grad,
                char* ws) {
  const size_t elems = (size_t)P->prob.n_rhs * P->state;
  const size_t lb = align_up(elems * sizeof(T));
  std::vector<T*> L(P->nmax + 1, nullptr);   // L[1..nmax]: forward levels of one sequence
  for (int s = 1; s <= P->nmax; ++s) L[s] = (T*)(ws + (size_t)(s - 1) * lb);
  T* bufA = (T*)(ws + (size_t)P->nmax * lb);
  T* bufB = (T*)(ws + (size_t)(P->nmax + 1) * lb);
  double* yacc = (double*)(ws + (size_t)(P->nmax + 2) * lb);
  double* facc = (double*)((char*)yacc + align_up(elems * 8));
  const unsigned gx = (unsigned)((P->field + 255) / 256);
  const unsigned gz = (unsigned)P->prob.n_rhs;
  hipStream_t s = P->stream;
  // the 3-D operator's z-marching sweeps unless a flat form is chosen
  const int v = resolve_variant(P);
  const bool march = OP == OP_AC3D && (v == GBS_VARIANT_MARCH8 || v == GBS_VARIANT_MARCH16 ||
                                      v == GBS_VARIANT_TILE3D);
  const unsigned mblocks = (unsigned)(((P->prob.n[0] + 63) / 64) * ((P->prob.n[1] + 3) / 4) *
                                      ((P->prob.n[2] + 63) / 64));
  // the LDS-tiled adjoint sweeps with the LDS-tiled forward form: 64 x 8
  // columns per block in FP64 (2 waves per SIMD), 64 x 12 in FP32 (3 waves:
  // one 768-thread block fills a CU; 64 x 8 blocks fit once per CU and
  // were slower than the z-marching sweeps)
  const bool tiled = OP == OP_AC3D && v == GBS_VARIANT_TILE3D;
  constexpr int ATZ = 128, ABY = sizeof(T) == 4 ? 12 : 8, AWPE = sizeof(T) == 4 ? 3 : 2;
  // planes per block of the tiled sweeps: a sweep runs its blocks in rounds
  // of the blocks the GPU holds at once (one per CU), so the z-chunking is
  // the one that minimises rounds x (planes + the 2R warm-up planes of a
  // chunk); 384^3 FP32: 96 planes (768 blocks, 3 rounds) rather than 128
  // (576 blocks: a third round a quarter full)
  unsigned tblocks = 0;
  int atz = ATZ;
  if (OP == OP_AC3D && tiled) {
    constexpr int RA = Fd<ORDER>::R;
    const long txy = (long)((P->prob.n[0] + 63) / 64) * (long)((P->prob.n[1] + ABY - 1) / ABY);
    const int nz = (int)P->prob.n[2];
    const int waves = resident_waves(adj_tile3d<T, ORDER, ATZ, ABY, false, true, AWPE>, 64 * ABY);
    const long slots = std::max(1, waves / ABY);
    double best = 1e300;
    int prev = 0;
    for (int m = 1; m <= std::max(1, nz / 16); ++m) {
      const int tz = (nz + m - 1) / m;
      if (tz == prev) continue;
      prev = tz;
      const long blocks = txy * ((nz + tz - 1) / tz);
      const double cost = (double)((blocks + slots - 1) / slots) * (double)(tz + 2 * RA);
      if (cost < best * (1.0 - 1e-9)) {
        best = cost;
        atz = tz;
      }
    }
    tblocks = (unsigned)(txy * ((nz + atz - 1) / atz));
  }

  if (tbar && P->nrec)
    hipLaunchKernelGGL(inject_kernel<T>, dim3((unsigned)((P->nrec + 255) / 256)), dim3(256), 0, s,
                       ybar, P->state, P->rec_dev, P->nrec, tbar, (int)P->rec_distinct);

  FirstArgs<T> fa;
  StepArgs<T> sa;
  std::memset(&fa, 0, sizeof(fa));
  std::memset(&sa, 0, sizeof(sa));
  fill_geometry<T>(P, fa.g, fa.c2c, fa.c2f, fa.invx, fa.invy, fa.invz);
  fill_geometry<T>(P, sa.g, sa.c2c, sa.c2f, sa.invx, sa.invy, sa.invz);
  std::memcpy(fa.src, P->src, sizeof(P->src));
  std::memcpy(sa.src, P->src, sizeof(P->src));
  AdjArgs<T> aa;
  std::memset(&aa, 0, sizeof(aa));
  T c2c_dummy;
  const T* c2f_dummy;
  fill_geometry<T>(P, aa.g, c2c_dummy, c2f_dummy, aa.invx, aa.invy, aa.invz);
  aa.c2f = c2f_dummy;
  aa.c2c = c2c_dummy;
  aa.ybar = ybar;
  aa.yacc = yacc;
  aa.facc = facc;
  aa.grad = grad;
  aa.nrhs = P->prob.n_rhs;
  aa.tz = atz;
  auto adj_sweep = [&](bool first) {
    if constexpr (OP == OP_AC3D) {
      if (tiled) {
        const dim3 g(tblocks), b(64 * ABY);
        if (first) {
          if (grad) hipLaunchKernelGGL((adj_tile3d<T, ORDER, ATZ, ABY, true, true, AWPE>), g, b, 0, s, aa);
          else hipLaunchKernelGGL((adj_tile3d<T, ORDER, ATZ, ABY, true, false, AWPE>), g, b, 0, s, aa);
        } else {
          if (grad) hipLaunchKernelGGL((adj_tile3d<T, ORDER, ATZ, ABY, false, true, AWPE>), g, b, 0, s, aa);
          else hipLaunchKernelGGL((adj_tile3d<T, ORDER, ATZ, ABY, false, false, AWPE>), g, b, 0, s, aa);
        }
        return;
      }
    }
    if (march) {
      if (first) hipLaunchKernelGGL((adj_march3d<T, ORDER, 64, true>), dim3(mblocks), dim3(256), 0, s, aa);
      else hipLaunchKernelGGL((adj_march3d<T, ORDER, 64, false>), dim3(mblocks), dim3(256), 0, s, aa);
    } else if (first) {
      hipLaunchKernelGGL((adj_first_kernel<T, ORDER, OP>), dim3(gx), dim3(256), 0, s, aa);
    } else {
      hipLaunchKernelGGL((adj_lf_kernel<T, ORDER, OP>), dim3(gx), dim3(256), 0, s, aa);
    }
  };

  for (int r = 0; r < P->k; ++r) {
    const int j = P->order[r];
    const int N = P->steps[j];
    const double h = P->H / N;
    // forward levels y_1..y_N of sequence j (y_0 is the input state)
    fa.y0 = y0;
    fa.nseq = 1;
    fa.out[0] = L[1];
    fa.h[0] = (T)h;
    fa.amp = P->nsrc ? ricker(t0, P->f0, P->delay) : 0.0;
    launch_first<T, ORDER, OP>(P, fa, gx, gz);
    for (int st = 1; st <= N - 1; ++st) {
      SeqDesc<T>& d = sa.seq[0];
      d.cur = L[st];
      d.old = st == 1 ? y0 : L[st - 1];
      d.out = L[st + 1];
      d.h2 = (T)(2.0 * h);
      d.cw = 0.0;
      d.amp = P->nsrc ? ricker(t0 + st * h, P->f0, P->delay) : 0.0;
      d.mode = 0;
      launch_lf<T, ORDER, OP>(P, sa, 1, gx, gz);
    }
    // transposed sequence
    aa.cw = P->w[j];
    aa.h = h;
    aa.first_seq = r == 0;
    aa.level = L[N];
    aa.P = bufA;
    aa.Q = bufB;
    aa.last = 0;
    adj_sweep(true);
    for (int n = N - 1; n >= 1; --n) {
      const bool a_is_p = ((N - 1 - n) % 2) == 0;
      aa.P = a_is_p ? bufA : bufB;
      aa.Q = a_is_p ? bufB : bufA;
      aa.level = n == 0 ? y0 : L[n];
      aa.last = n == 1;
      adj_sweep(false);
    }
  }
  AdjFinalArgs<T> fz;
  std::memset(&fz, 0, sizeof(fz));
  T ix, iy, iz;
  fill_geometry<T>(P, fz.g, fz.c2c, fz.c2f, ix, iy, iz);
  const double den = P->prob.fd_order == 8 ? 840.0 : 12.0;
  fz.invx = (double)P->prob.n[0] / den;
  fz.invy = (double)P->prob.n[1] / den;
  fz.invz = (double)P->prob.n[2] / den;
  fz.yacc = yacc;
  fz.facc = facc;
  fz.y0 = y0;
  fz.ybar = ybar;
  fz.grad = grad;
  fz.nrhs = P->prob.n_rhs;
  hipLaunchKernelGGL((adj_final_kernel<T, ORDER, OP>), dim3(gx), dim3(256), 0, s, fz);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return fail(GBS_EDEVICE, "kernel launch failed: %s", hipGetErrorString(e));
  return GBS_OK;
}

template <typename T>
int adjoint_dispatch(gbs_plan* P, double t0, const void* y0, void* ybar, const void* tbar,
                     double* grad, char* ws) {
  const T* a = (const T*)y0;
  T* b = (T*)ybar;
  const T* c = (const T*)tbar;
  if (blocked_adjoint(P)) return adjoint_blocked_run<T>(P, t0, a, b, c, grad, ws);
  if (P->prob.fd_order == 4) {
    if (P->prob.op == GBS_ACOUSTIC2D) return adjoint_run<T, 4, OP_AC2D>(P, t0, a, b, c, grad, ws);
    return adjoint_run<T, 4, OP_AC3D>(P, t0, a, b, c, grad, ws);
  }
  if (P->prob.op == GBS_ACOUSTIC2D) return adjoint_run<T, 8, OP_AC2D>(P, t0, a, b, c, grad, ws);
  return adjoint_run<T, 8, OP_AC3D>(P, t0, a, b, c, grad, ws);
}

}  // namespace

extern "C" int gbs_plan_adjoint_workspace_bytes(const gbs_plan* P, size_t* bytes) {
  if (!P || !bytes) return fail(GBS_EINVAL, "null argument");
  *bytes = adjoint_bytes(P);
  return GBS_OK;
}

namespace {

int check_adjoint_args(const gbs_plan* P, double t0, const void* y_in, const void* ybar,
                       double* grad_c2, const void* adj_ws, size_t adj_ws_bytes) {
  if (!P || !y_in || !ybar || !adj_ws) return fail(GBS_EINVAL, "null argument");
  if (P->prob.op == GBS_ADVECT1D) return fail(GBS_EUNSUPPORTED, "the adjoint is built for the acoustic operators");
  if (grad_c2 && !P->prob.c2_field)
    return fail(GBS_EINVAL, "a c^2 gradient needs a plan with a coefficient field");
  if ((uintptr_t)adj_ws % kAlign) return fail(GBS_EINVAL, "adjoint workspace must be 256-byte aligned");
  if (adj_ws_bytes < adjoint_bytes(P))
    return fail(GBS_ENOMEM, "adjoint workspace has %zu bytes, needs %zu", adj_ws_bytes,
                adjoint_bytes(P));
  if (!std::isfinite(t0)) return fail(GBS_EINVAL, "t0 must be finite");
  return GBS_OK;
}

}  // namespace

extern "C" int gbs_adjoint_step(gbs_plan* P, double t0, const void* y_in, void* ybar,
                                const void* trace_bar, double* grad_c2, void* adj_ws,
                                size_t adj_ws_bytes) {
  const int st = check_adjoint_args(P, t0, y_in, ybar, grad_c2, adj_ws, adj_ws_bytes);
  if (st) return st;
  if (P->prob.dtype == GBS_F64)
    return adjoint_dispatch<double>(P, t0, y_in, ybar, trace_bar, grad_c2, (char*)adj_ws);
  return adjoint_dispatch<float>(P, t0, y_in, ybar, trace_bar, grad_c2, (char*)adj_ws);
}

extern "C" int gbs_step_keep_pairs(gbs_plan* P, double t0, int32_t n_macro, const void* y_in,
                                   void* y_out, void* pairs) {
  if (!P || !y_in || !y_out || !pairs) return fail(GBS_EINVAL, "null argument");
  if (n_macro < 1) return fail(GBS_EINVAL, "n_macro must be >= 1");
  if (!blocked_adjoint(P))
    return fail(GBS_EUNSUPPORTED,
                "kept pairs need the 2-D FD4 operator with a temporally blocked variant");
  P->keep_out = pairs;
  const int st = gbs_step(P, t0, n_macro, y_in, y_out);
  P->keep_out = nullptr;
  return st;
}

extern "C" int gbs_adjoint_step_pairs(gbs_plan* P, double t0, const void* y_in,
                                      const void* pairs, void* ybar, const void* trace_bar,
                                      double* grad_c2, void* adj_ws, size_t adj_ws_bytes) {
  int st = check_adjoint_args(P, t0, y_in, ybar, grad_c2, adj_ws, adj_ws_bytes);
  if (st) return st;
  if (!pairs) return fail(GBS_EINVAL, "null argument");
  if (!blocked_adjoint(P))
    return fail(GBS_EUNSUPPORTED,
                "kept pairs need the 2-D FD4 operator with a temporally blocked variant");
  if (P->prob.dtype == GBS_F64)
    return adjoint_blocked_run<double>(P, t0, (const double*)y_in, (double*)ybar,
                                       (const double*)trace_bar, grad_c2, (char*)adj_ws,
                                       (const double*)pairs);
  return adjoint_blocked_run<float>(P, t0, (const float*)y_in, (float*)ybar,
                                    (const float*)trace_bar, grad_c2, (char*)adj_ws,
                                    (const float*)pairs);
}
