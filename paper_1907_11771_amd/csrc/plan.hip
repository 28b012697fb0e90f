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
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "internal.hpp"
#include "kernels.hpp"
#include "temporal.hpp"

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
  // sources
  int nsrc = 0;
  SrcDesc src[GBS_MAX_SRC];
  double f0 = 0, delay = 0;
  // leap-frog kernel variant (GBS_VARIANT_*) and rows per band of the
  // temporally blocked passes
  int variant = 0;
  int band = 64;
  // temporally blocked layout: per sequence two pairs of levels
  void* pair[GBS_MAX_SEQ][2][2];
  // timing
  bool timing = false;
  std::vector<EventPair> lf_ev, first_ev;
  size_t lf_used = 0, first_used = 0;
};

namespace {

constexpr size_t kAlign = 256;
size_t align_up(size_t v) { return (v + kAlign - 1) / kAlign * kAlign; }

int fields_of(int op) {
  return op == GBS_ADVECT1D ? 1 : (op == GBS_ACOUSTIC2D ? 3 : (op == GBS_ACOUSTIC3D ? 4 : 0));
}
int dims_of(int op) { return op == GBS_ADVECT1D ? 1 : (op == GBS_ACOUSTIC2D ? 2 : 3); }
size_t dsize(int dtype) { return dtype == GBS_F32 ? 4 : 8; }

int validate_problem(const gbs_problem* p) {
  if (!p) return fail(GBS_EINVAL, "problem is null");
  if (!fields_of(p->op)) return fail(GBS_EINVAL, "unknown operator %d", p->op);
  if (p->fd_order != 4 && p->fd_order != 8) return fail(GBS_EUNSUPPORTED, "fd_order must be 4 or 8");
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

size_t workspace_bytes(const gbs_problem* p, int k) {
  const int64_t pts = p->n[0] * p->n[1] * p->n[2];
  const size_t elems = (size_t)p->n_rhs * fields_of(p->op) * pts;
  return align_up(elems * 8) + levels_per_seq(p) * (size_t)k * align_up(elems * dsize(p->dtype));
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
  const double den = P->prob.fd_order == 8 ? 840.0 : 12.0;
  ix = (T)((double)P->prob.n[0] / den);
  iy = (T)((double)P->prob.n[1] / den);
  iz = (T)((double)P->prob.n[2] / den);
  c2c = (T)(P->prob.op == GBS_ADVECT1D ? 1.0 : P->prob.c2);
  c2f = (const T*)P->prob.c2_field;
}

int resolve_variant(const gbs_plan* P) {
  if (P->variant != GBS_VARIANT_AUTO) return P->variant;
  if (P->prob.op == GBS_ACOUSTIC2D) return GBS_VARIANT_TEMPORAL;
  return GBS_VARIANT_FLAT;
}

bool is_temporal(int v) { return v >= GBS_VARIANT_TEMPORAL && v <= GBS_VARIANT_TEMPORAL_S6; }

template <typename T, int ORDER, int G, bool SKEW1>
int run_temporal(gbs_plan* P, double t0, int n_macro, const T* yin, T* yout) {
  constexpr int R = Fd<ORDER>::R;
  // split the N_j + 1 evaluations of every sequence into passes of at most G
  int npass[GBS_MAX_SEQ], gsz[GBS_MAX_SEQ][32];
  int maxpass = 0;
  for (int j = 0; j < P->k; ++j) {
    const int E = P->steps[j] + 1;
    const int np = (E + G - 1) / G;
    if (np > 32) return fail(GBS_EUNSUPPORTED, "too many passes");
    npass[j] = np;
    for (int q = 0; q < np; ++q) gsz[j][q] = E / np + (q < E % np ? 1 : 0);
    maxpass = std::max(maxpass, np);
  }
  PassArgs<T> pa;
  std::memset(&pa, 0, sizeof(pa));
  T c2c, invz;
  fill_geometry<T>(P, pa.g, c2c, pa.c2f, pa.invx, pa.invy, invz);
  pa.c2c = c2c;
  std::memcpy(pa.src, P->src, sizeof(P->src));
  pa.band = P->band;
  pa.nbands = (int)((P->prob.n[1] + P->band - 1) / P->band);
  const int nx = (int)P->prob.n[0];
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
  for (int m = 0; m < n_macro; ++m) {
    const double t = t0 + m * P->H;
    const T* y0 = m == 0 ? yin : yout;
    for (int q = 0; q < maxpass; ++q) {
      int n = 0, maxs = 0;
      for (int r = 0; r < P->k; ++r) {
        const int j = P->order[r];
        if (q >= npass[j]) continue;
        PassSeq<T>& d = pa.seq[n++];
        const double h = P->H / P->steps[j];
        int s0 = 0;             // the pass's input level is y_{s0}: s0 = evaluations so far
        for (int qq = 0; qq < q; ++qq) s0 += gsz[j][qq];
        d.g = gsz[j][q];
        d.h = (T)h;
        d.flags = (q == 0 ? PASS_FIRST : 0) | (q == npass[j] - 1 ? PASS_FINAL : 0);
        d.cur = q == 0 ? y0 : (const T*)P->pair[j][(q - 1) % 2][1];
        d.old = q == 0 ? nullptr : (const T*)P->pair[j][(q - 1) % 2][0];
        d.out_a = (T*)P->pair[j][q % 2][0];
        d.out_b = (T*)P->pair[j][q % 2][1];
        d.ystar = (double*)P->pair[j][q % 2][0];
        d.strips = (nx + (64 - 2 * d.g * R) - 1) / (64 - 2 * d.g * R);
        for (int e = 0; e < d.g; ++e)
          d.amp[e] = P->nsrc ? ricker(t + (s0 + e) * h, P->f0, P->delay) : 0.0;
        maxs = std::max(maxs, d.strips);
      }
      pa.max_strips = maxs;
      const unsigned waves = (unsigned)maxs * pa.nbands;
      EventPair* ev = nullptr;
      if (P->timing) {
        ev = &next_event(P->lf_ev, P->lf_used);
        hipEventRecord(ev->a, P->stream);
      }
      hipLaunchKernelGGL((pass2d<T, ORDER, G, SKEW1>), dim3((waves + 3) / 4, n, P->prob.n_rhs),
                         dim3(256), 0, P->stream, pa);
      if (ev) hipEventRecord(ev->b, P->stream);
    }
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

template <typename T, int ORDER, int OP>
void launch_lf(gbs_plan* P, const StepArgs<T>& sa, int n, unsigned gx, unsigned gz) {
  if constexpr (OP == OP_AC2D) {
    switch (resolve_variant(P)) {
      case GBS_VARIANT_MARCH8: launch_march2d<T, ORDER, 8, false>(P, sa, n, gz); return;
      case GBS_VARIANT_MARCH16: launch_march2d<T, ORDER, 16, false>(P, sa, n, gz); return;
      case GBS_VARIANT_MARCH8_NT: launch_march2d<T, ORDER, 8, true>(P, sa, n, gz); return;
      case GBS_VARIANT_MARCH16_NT: launch_march2d<T, ORDER, 16, true>(P, sa, n, gz); return;
      default: break;
    }
  }
  hipLaunchKernelGGL((lf_kernel<T, ORDER, OP>), dim3(gx, n, gz), dim3(256), 0, P->stream, sa);
}

template <typename T, int ORDER, int OP>
int run(gbs_plan* P, double t0, int n_macro, const T* yin, T* yout) {
  const int block = 256;
  const unsigned gx = (unsigned)((P->field + block - 1) / block);
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
    hipLaunchKernelGGL((first_kernel<T, ORDER, OP>), dim3(gx, 1, gz), dim3(block), 0, P->stream, fa);
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

template <typename T>
int dispatch_order(gbs_plan* P, double t0, int n, const void* yin, void* yout) {
  const T* a = (const T*)yin;
  T* b = (T*)yout;
  const int op = P->prob.op;
  const int v = resolve_variant(P);
  if (op == GBS_ACOUSTIC2D && is_temporal(v)) {
    if (P->prob.fd_order == 8) return run_temporal<T, 8, 3, true>(P, t0, n, a, b);
    switch (v) {
      case GBS_VARIANT_TEMPORAL4: return run_temporal<T, 4, 4, false>(P, t0, n, a, b);
      case GBS_VARIANT_TEMPORAL_S5: return run_temporal<T, 4, 5, true>(P, t0, n, a, b);
      case GBS_VARIANT_TEMPORAL_S6: return run_temporal<T, 4, 6, true>(P, t0, n, a, b);
      default: return run_temporal<T, 4, 7, false>(P, t0, n, a, b);
    }
  }
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

extern "C" int gbs_plan_create(gbs_plan** out, const gbs_problem* prob, const gbs_scheme* sch,
                               double H, void* workspace, size_t ws_bytes, void* hip_stream) {
  try {
    if (!out) return fail(GBS_EINVAL, "out is null");
    *out = nullptr;
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
    if (!(prob->flags & GBS_FLAG_NO_STABILITY_CHECK)) {
      std::vector<Rational> c(sch->k);
      for (int j = 0; j < sch->k; ++j) c[j] = Rational::from_double(sch->weights[j]);
      const double isb = isb_of(sch->k, sch->steps, c);
      const int d = dims_of(prob->op);
      double s2 = 0;
      for (int a = 0; a < d; ++a) s2 += (double)prob->n[a] * (double)prob->n[a];
      const double cmax = prob->op == GBS_ADVECT1D
                              ? 1.0
                              : (prob->c2_field ? prob->c_max : std::sqrt(prob->c2));
      const double rho = cmax * stencil_sigma(prob->fd_order) * std::sqrt(s2);
      if (H * rho > isb)
        return fail(GBS_EUNSTABLE, "H * rho = %.6g exceeds the scheme's ISB %.6g", H * rho, isb);
    }
    gbs_plan* P = new gbs_plan();
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
    *out = P;
    return GBS_OK;
  } catch (const std::exception& e) {
    return fail(GBS_EINVAL, "gbs_plan_create: %s", e.what());
  }
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
  if (P->prob.dtype == GBS_F64) return dispatch_order<double>(P, t0, n_macro, y_in, y_out);
  return dispatch_order<float>(P, t0, n_macro, y_in, y_out);
}

extern "C" int gbs_plan_set_variant(gbs_plan* P, int32_t variant) {
  if (!P) return fail(GBS_EINVAL, "plan is null");
  if (variant < GBS_VARIANT_AUTO || variant > GBS_VARIANT_TEMPORAL_S6)
    return fail(GBS_EINVAL, "unknown variant %d", variant);
  if (variant >= GBS_VARIANT_MARCH8 && P->prob.op != GBS_ACOUSTIC2D)
    return fail(GBS_EUNSUPPORTED, "this variant is built for the 2-D acoustic operator only");
  P->variant = variant;
  return GBS_OK;
}

extern "C" int gbs_plan_set_band(gbs_plan* P, int32_t rows) {
  if (!P) return fail(GBS_EINVAL, "plan is null");
  if (rows < 1 || rows > (1 << 20)) return fail(GBS_EINVAL, "rows per band out of range");
  P->band = rows;
  return GBS_OK;
}

extern "C" int gbs_plan_get_variant(const gbs_plan* P, int32_t* variant) {
  if (!P || !variant) return fail(GBS_EINVAL, "null argument");
  *variant = resolve_variant(P);
  return GBS_OK;
}

extern "C" int gbs_plan_set_timing(gbs_plan* P, int32_t enabled) {
  if (!P) return fail(GBS_EINVAL, "plan is null");
  if (enabled < 0) return fail(GBS_EINVAL, "enabled must be >= 0");
  P->timing = enabled != 0;
  P->lf_used = P->first_used = 0;
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
// in use: every level or accumulator a kernel must read or write once over
// the grid (halo re-reads and redundant edge work are not counted).
extern "C" int gbs_plan_algorithmic_bytes(const gbs_plan* P, double* step_bytes,
                                          int64_t* step_launches, double* aux_bytes,
                                          int64_t* aux_launches) {
  if (!P) return fail(GBS_EINVAL, "plan is null");
  const double pts = (double)P->field * P->prob.n_rhs;
  const double Fb = (double)P->F * dsize(P->prob.dtype);   // one level, per point
  const double F8 = (double)P->F * 8.0;                     // one FP64 state, per point
  const int v = resolve_variant(P);
  double sb = 0, ab = 0;
  int64_t sl = 0, al = 0;
  if (P->prob.op == GBS_ACOUSTIC2D && is_temporal(v)) {
    const int G = v == GBS_VARIANT_TEMPORAL4 ? 4 : v == GBS_VARIANT_TEMPORAL_S5 ? 5
                : v == GBS_VARIANT_TEMPORAL_S6 ? 6 : (P->prob.fd_order == 8 ? 3 : 7);
    const int Gx = P->prob.fd_order == 8 ? 3 : G;
    int maxpass = 0;
    for (int j = 0; j < P->k; ++j) {
      const int E = P->steps[j] + 1, np = (E + Gx - 1) / Gx;
      maxpass = std::max(maxpass, np);
      for (int q = 0; q < np; ++q) {
        sb += (q == 0 ? Fb : 2 * Fb) * pts;                  // inputs
        sb += (q == np - 1 ? F8 : 2 * Fb) * pts;             // outputs
      }
    }
    sl = maxpass;
    ab = ((double)P->k * F8 + Fb) * pts;                     // combine
    al = 1;
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
    ab = (1 + P->k) * Fb * pts;                              // first evaluation
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

extern "C" int gbs_plan_destroy(gbs_plan* P) {
  if (!P) return GBS_OK;
  for (auto& e : P->lf_ev) { hipEventDestroy(e.a); hipEventDestroy(e.b); }
  for (auto& e : P->first_ev) { hipEventDestroy(e.a); hipEventDestroy(e.b); }
  delete P;
  return GBS_OK;
}

extern "C" const char* gbs_last_error(void) { return g_last_error.c_str(); }
