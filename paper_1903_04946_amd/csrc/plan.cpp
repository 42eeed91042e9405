// plan.cpp -- host planner and the C ABI of libsoprop (see include/soprop.h).
//
// The planner turns a scheme (splitting, composition, order) into the pruned
// action sequence with unique coefficients (Sec. "Symmetric composition
// schemes", Sec. "Pruning splitting coefficients", Table II), uploads the
// V-table, forms the unique potential tables on the device, computes the
// per-axis kinetic factors and FFT twiddles in extended precision, and
// drives the kernels.  It shares no code with the CPU oracle.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>
#include <algorithm>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "../../include/soprop.h"
#include "fft_core.hpp"
#include "internal.hpp"

using sop::DevView;

namespace {

thread_local std::string g_err;

sop_status fail(sop_status s, const std::string& msg) {
  g_err = msg;
  return s;
}

#define HIPTRY(expr)                                                                 \
  do {                                                                               \
    hipError_t _e = (expr);                                                          \
    if (_e != hipSuccess) {                                                          \
      return fail(SOP_ERR_HIP, std::string(#expr) + ": " + hipGetErrorString(_e));   \
    }                                                                                \
  } while (0)

typedef long double ld;
const ld kTwoPi = 6.283185307179586476925286766559005768394L;

// ------------------------------------------------------------------ schemes
// Outer coefficients of one recursion level raising the order p -> p+2:
// triple jump (c, 1-2c, c), c = 1/(2 - 2^(1/(p+1))); Suzuki's fractal
// (c, c, 1-4c, c, c), c = 1/(4 - 4^(1/(p+1))).
std::vector<ld> level_coefficients(sop_comp comp, int p) {
  if (comp == SOP_COMP_TRIPLE_JUMP) {
    const ld c = 1.0L / (2.0L - std::pow(2.0L, 1.0L / (ld)(p + 1)));
    return {c, 1.0L - 2.0L * c, c};
  }
  const ld c = 1.0L / (4.0L - std::pow(4.0L, 1.0L / (ld)(p + 1)));
  return {c, c, 1.0L - 4.0L * c, c, c};
}

// Composition coefficients gamma_0..gamma_{M-1}.  Stage i of the flattened
// recursion is the product over levels of the level's coefficient picked by
// the base-3 (or base-5) digit of i; the least significant digit belongs to
// the innermost level (order 2 -> 4), since every outer stage scales a whole
// inner sequence.
bool composition(sop_comp comp, int order, std::vector<ld>& g) {
  g.clear();
  if (comp == SOP_COMP_STRANG) {
    if (order != 2) return false;
    g.push_back(1.0L);
    return true;
  }
  if (comp != SOP_COMP_TRIPLE_JUMP && comp != SOP_COMP_SUZUKI) return false;
  if (order < 2 || order > 10 || (order & 1)) return false;
  const int levels = order / 2 - 1;
  const int base = comp == SOP_COMP_TRIPLE_JUMP ? 3 : 5;
  std::vector<std::vector<ld>> lc;
  for (int l = 0; l < levels; ++l) lc.push_back(level_coefficients(comp, 2 * l + 2));
  int M = 1;
  for (int l = 0; l < levels; ++l) M *= base;
  g.resize(M);
  for (int i = 0; i < M; ++i) {
    ld prod = 1.0L;
    int r = i;
    for (int l = 0; l < levels; ++l) {
      prod *= lc[l][r % base];
      r /= base;
    }
    g[i] = prod;
  }
  return true;
}

struct Sequence {
  int M = 0;                   // number of B actions
  std::vector<double> a, b;    // pruned sequence, a has M+1 entries (1 for VT/TV)
  std::vector<double> au, bu;  // unique values
  std::vector<int> ia, ib;     // indices (ib has M entries)
  std::vector<double> g;       // composition coefficients (empty for VT/TV)
  bool a_is_v = true;
};

// Unique values of a palindromic list, searching only its first half and
// mirroring the indices (symmetry, Eq. symmetric_splitting_coefficients).
void unique_palindrome(const std::vector<double>& v, std::vector<double>& unq,
                       std::vector<int>& idx) {
  const int n = (int)v.size();
  unq.clear();
  idx.assign(n, -1);
  for (int j = 0; j < (n + 1) / 2; ++j) {
    int hit = -1;
    for (int u = 0; u < (int)unq.size() && hit < 0; ++u) {
      const double tol = 1e-13 * std::fmax(std::fabs(v[j]), std::fabs(unq[u]));
      if (std::fabs(v[j] - unq[u]) <= tol) hit = u;
    }
    if (hit < 0) {
      unq.push_back(v[j]);
      hit = (int)unq.size() - 1;
    }
    idx[j] = hit;
    idx[n - 1 - j] = hit;
  }
}

// Largest number of Strang stages a custom composition may have (Suzuki's
// tenth order, the longest built-in scheme, has 625).
constexpr int kMaxCustomStages = 625;

// Caller-supplied composition coefficients (Sec. "Symmetric composition
// schemes": a composition of Strang stages with coefficients gamma_1..gamma_M
// that sum to one, symmetric under j -> M+1-j so that the composed method is
// symmetric).  Symmetry is required because the unique-coefficient search
// covers only the first half of the sequence.
sop_status custom_composition(int M, const double* gamma, std::vector<ld>& g) {
  if (!gamma) return fail(SOP_ERR_INVALID, "a custom composition needs gamma");
  if (M < 1 || M > kMaxCustomStages)
    return fail(SOP_ERR_INVALID, "custom composition: ngamma must be 1.." +
                                     std::to_string(kMaxCustomStages));
  double gmax = 0;
  ld sum = 0;
  for (int j = 0; j < M; ++j) {
    if (!std::isfinite(gamma[j]) || gamma[j] == 0)
      return fail(SOP_ERR_INVALID, "custom composition: every gamma must be finite and nonzero");
    gmax = std::fmax(gmax, std::fabs(gamma[j]));
    sum += gamma[j];
  }
  for (int j = 0; j < M / 2; ++j)
    if (std::fabs(gamma[j] - gamma[M - 1 - j]) > 1e-14 * gmax)
      return fail(SOP_ERR_INVALID, "custom composition: gamma must be symmetric (gamma_j = gamma_{M+1-j})");
  if (std::fabs((double)(sum - 1.0L)) > 1e-12 * std::fmax(1.0, gmax))
    return fail(SOP_ERR_INVALID, "custom composition: gamma must sum to 1");
  g.assign(gamma, gamma + M);
  // mirror exactly, so that the pruned sequence is an exact palindrome
  for (int j = 0; j < M / 2; ++j) g[M - 1 - j] = g[j];
  return SOP_OK;
}

sop_status build_sequence(sop_split split, sop_comp comp, int order, int ngamma,
                          const double* gamma, Sequence& s) {
  s = Sequence();
  if (split == SOP_SPLIT_VT || split == SOP_SPLIT_TV) {
    if (order != 1 || comp != SOP_COMP_STRANG)
      return fail(SOP_ERR_INVALID, "first-order splittings take comp = STRANG and order = 1");
    s.M = 1;
    s.a = {1.0};
    s.b = {1.0};
    s.au = {1.0};
    s.bu = {1.0};
    s.ia = {0};
    s.ib = {0};
    s.a_is_v = (split == SOP_SPLIT_TV);  // TV applies V first
    return SOP_OK;
  }
  if (split != SOP_SPLIT_VTV && split != SOP_SPLIT_TVT)
    return fail(SOP_ERR_INVALID, "unknown splitting");
  if (comp != SOP_COMP_CUSTOM && (ngamma != 0 || gamma))
    return fail(SOP_ERR_INVALID, "gamma is given only with comp = SOP_COMP_CUSTOM");
  std::vector<ld> g;
  if (comp == SOP_COMP_CUSTOM) {
    if (order < 2 || (order & 1))
      return fail(SOP_ERR_INVALID, "custom composition: order (the stated order) must be even and >= 2");
    const sop_status st = custom_composition(ngamma, gamma, g);
    if (st != SOP_OK) return st;
  } else if (!composition(comp, order, g)) {
    return fail(SOP_ERR_INVALID, "invalid composition/order (Strang: 2; TJ/SF: 2..10 even)");
  }
  const int M = (int)g.size();
  s.M = M;
  s.g.assign(g.begin(), g.end());
  // Pruned sequence (Eq. merging_splitting_coeff_b_zero applied to every
  // Strang stage A(g/2) B(g) A(g/2)): a_1 = g_1/2, a_j = (g_{j-1} + g_j)/2,
  // a_{M+1} = g_M/2 and b_j = g_j.
  s.a.resize(M + 1);
  s.b.resize(M);
  s.a[0] = (double)(g[0] / 2);
  for (int j = 1; j < M; ++j) s.a[j] = (double)((g[j - 1] + g[j]) / 2);
  s.a[M] = (double)(g[M - 1] / 2);
  for (int j = 0; j < M; ++j) s.b[j] = (double)g[j];
  unique_palindrome(s.a, s.au, s.ia);
  unique_palindrome(s.b, s.bu, s.ib);
  s.a_is_v = (split == SOP_SPLIT_VTV);
  return SOP_OK;
}

bool supported_length(int ndim, int n) {
  if (ndim == 1) return sop::k1d_supported(n, 1);
  if (ndim == 3) return sop::k3d_supported(n, 1);
  return false;
}

}  // namespace

// ------------------------------------------------------------------ plan
struct sop_plan {
  int ndim = 1;
  int n[3] = {1, 1, 1};
  double lo[3] = {0, 0, 0}, hi[3] = {1, 1, 1}, dx[3] = {1, 1, 1};
  double inv_mass[3] = {0, 0, 0};
  int S = 1;
  int64_t npts = 1;
  double dt = 0, hbar = 1, dV = 1;
  sop_dtype dtype = SOP_C128;
  size_t csize = 16;  // bytes per complex element
  Sequence seq;
  std::vector<double> vtaus;  // c dt / hbar of the potential tables
  std::vector<double> ttaus;  // c dt of the kinetic factor sets
  DevView dv;
  double* d_vraw = nullptr;
  void* d_vexp = nullptr;
  void* d_kin = nullptr;
  void* d_tw = nullptr;
  int* d_prog = nullptr;
  int* d_prog1 = nullptr;  // single-action programs {V(0), T(0)}
  double* d_taus = nullptr;
  void* d_scratch = nullptr;
  void* d_trap = nullptr;  // trapezoidal rule: residual, stats, stage taus
  size_t trap_bytes = 0;
  void* d_iws = nullptr;  // sop_interpolate workspace (grown on demand)
  size_t iws_bytes = 0;
  double iws_key[9] = {0};  // source grid whose axis matrices the workspace holds
  bool iws_valid = false;
  void* d_atab = nullptr;  // table for sop_apply_action
  void* d_akin = nullptr;
  double* d_part = nullptr;
  double* d_out = nullptr;
  size_t table_bytes = 0;
  bool eig_form = false;  // d_vexp holds the compact eigen form (3D FP64, S >= 2)
  double vbound = 0;      // max over points of max_i sum_j |V_ij| (bounds |lam|)
  std::vector<double> dvbound;  // the same for each dvtables[k]
  int tile = 0;  // potential-table layout (0 = [u][entry][point])
  sop::Timer* timer = nullptr;
  int nparams = 0;
  double* d_vbase = nullptr;  // V at theta = 0
  double* d_dv = nullptr;     // [nparams][NE][npts]
  double* d_theta = nullptr;  // [nparams]
  std::vector<double> theta;  // host copy of the current parameters
  double* d_drive = nullptr;  // drive samples of sop_propagate_driven
  size_t drive_cap = 0;       // doubles held by d_drive
  void* d_eig = nullptr;      // adjoint eigen table (FP64, tile layout)
  double* d_w = nullptr;      // [S] adjoint weights
  sop::GraphCache* graphs = nullptr;
  bool use_graphs = true;
  // captured blocks of 3D trapezoidal iterations, keyed by state, workspace
  // and stage coefficient (the kernels' pointers and tau)
  struct T3Key {
    const void* x;
    const void* base;
    uint64_t tau;
    bool operator<(const T3Key& o) const {
      if (x != o.x) return x < o.x;
      if (base != o.base) return base < o.base;
      return tau < o.tau;
    }
  };
  std::map<T3Key, hipGraphExec_t> t3graphs;
  sop_allocator hook{};  // device memory hooks (alloc == NULL: hipMalloc/hipFree)
  hipStream_t home = nullptr;  // the creation stream, handed to the hooks
};

namespace sop {
const DevView* plan_view(const sop_plan* p) { return &p->dv; }
void set_last_error(const std::string& msg) { g_err = msg; }
}  // namespace sop

namespace {

// Device buffers of a plan: through the caller's hooks when given.
hipError_t dalloc(sop_plan* p, void** ptr, size_t bytes) {
  if (p->hook.alloc) {
    *ptr = p->hook.alloc(p->hook.ctx, bytes, (void*)p->home);
    return *ptr ? hipSuccess : hipErrorOutOfMemory;
  }
  return hipMalloc(ptr, bytes);
}
template <typename T>
hipError_t dalloc(sop_plan* p, T** ptr, size_t bytes) {
  void* v = nullptr;
  const hipError_t e = dalloc(p, &v, bytes);
  *ptr = (T*)v;
  return e;
}

void free_plan(sop_plan* p) {
  if (!p) return;
  void* bufs[] = {p->d_vraw, p->d_vexp, p->d_kin, p->d_tw, p->d_prog, p->d_prog1, p->d_taus,
                  p->d_scratch, p->d_atab, p->d_akin, p->d_part, p->d_out, p->d_vbase,
                  p->d_dv, p->d_theta, p->d_eig, p->d_w, p->d_drive, p->d_iws, p->d_trap};
  delete p->graphs;
  for (auto& kv : p->t3graphs) (void)hipGraphExecDestroy(kv.second);
  for (void* b : bufs) {
    if (!b) continue;
    if (p->hook.free)
      p->hook.free(p->hook.ctx, b, (void*)p->home);
    else
      (void)hipFree(b);
  }
  delete p->timer;
  delete p;
}

// Kinetic factors of one coefficient set: [ntau][ndim or 3][n] complex,
// f_d(k) = exp(-i tau hbar kappa_k^2 inv_mass_d / 2) / n_d; every axis
// carries the 1/n_d of its own unnormalised inverse transform.
std::vector<ld> kinetic_factors(const sop_plan* p, const std::vector<double>& taus) {
  const int nax = p->ndim == 1 ? 1 : 3;
  const int nn = p->n[0];
  std::vector<ld> out((size_t)taus.size() * nax * nn * 2);
  for (size_t u = 0; u < taus.size(); ++u)
    for (int a = 0; a < nax; ++a)
      for (int k = 0; k < nn; ++k) {
        const int kk = (k < nn / 2) ? k : k - nn;
        const ld kap = kTwoPi * (ld)kk / ((ld)p->n[a] * (ld)p->dx[a]);
        const ld ph = -(ld)taus[u] * (ld)p->hbar * kap * kap * (ld)p->inv_mass[a] / 2.0L;
        const size_t o = (((size_t)u * nax + a) * nn + k) * 2;
        const ld scale = 1.0L / (ld)p->n[a];
        out[o] = std::cos(ph) * scale;
        out[o + 1] = std::sin(ph) * scale;
      }
  return out;
}

// Largest Gershgorin row sum of a packed [S(S+1)/2][npts] symmetric table: a
// bound on every |eigenvalue| at every point.
double gershgorin_bound(const double* v, int S, int64_t npts) {
  std::vector<int> idx((size_t)S * S);
  int e = 0;
  for (int i = 0; i < S; ++i)
    for (int j = i; j < S; ++j) {
      idx[(size_t)i * S + j] = e;
      idx[(size_t)j * S + i] = e;
      ++e;
    }
  double b = 0.0;
  for (int64_t x = 0; x < npts; ++x)
    for (int i = 0; i < S; ++i) {
      double r = 0.0;
      for (int j = 0; j < S; ++j) r += std::fabs(v[(int64_t)idx[(size_t)i * S + j] * npts + x]);
      b = std::max(b, r);
    }
  return b;
}

// Whether every phase the eigen-form z-pass forms, tau lam with tau up to
// twice the largest coefficient (two merged actions) or `extra_tau`, stays
// within the range of its phase routine.
bool phases_fit(const sop_plan* p, double vbound, double extra_tau = 0.0) {
  double tmax = std::fabs(extra_tau);
  for (double t : p->vtaus) tmax = std::max(tmax, 2.0 * std::fabs(t));
  return tmax * vbound <= sop::kPhaseMax;
}

// Bound on |lam| of V = V0 + sum_k theta_k D_k from the bound of V0.
double param_bound(const sop_plan* p, double v0bound, const double* theta) {
  double b = v0bound;
  for (int k = 0; k < p->nparams; ++k) b += std::fabs(theta[k]) * p->dvbound[k];
  return b;
}

// Forms the potential tables of the plan from its raw V-table on the device:
// the compact eigen form, or one exp(-i tau V) table per unique coefficient.
hipError_t form_tables(sop_plan* p) {
  if (p->eig_form) return sop::form_eigq(p->dv, p->d_vraw, p->tile, p->d_vexp);
  return sop::form_vexp(p->dv, p->d_vraw, p->d_taus, (int)p->vtaus.size(), p->tile, p->d_vexp);
}

// Rounds blocks of n interleaved extended-precision complex values to the
// plan precision.  In FP32 each value becomes the pair (rounded, residue =
// value - rounded), which the FP32 kernels fold into their products with
// these factors.
std::vector<char> pack_split(const std::vector<ld>& v, bool f64, int n) {
  if (f64) {
    std::vector<char> out(v.size() * sizeof(double));
    double* d = reinterpret_cast<double*>(out.data());
    for (size_t i = 0; i < v.size(); ++i) d[i] = (double)v[i];
    return out;
  }
  const size_t nb = v.size() / (2 * (size_t)n);
  std::vector<char> out(nb * (size_t)n * 4 * sizeof(float));
  float* f = reinterpret_cast<float*>(out.data());
  for (size_t b = 0; b < nb; ++b)
    for (int k = 0; k < n; ++k)
      for (int c = 0; c < 2; ++c) {
        const ld x = v[(b * n + k) * 2 + c];
        const float hi = (float)(double)x;
        f[((b * n + k) * 2) * 2 + c] = hi;
        f[((b * n + k) * 2 + 1) * 2 + c] = (float)(double)(x - (ld)hi);
      }
  return out;
}

sop_status validate(const sop_plan_desc* d) {
  if (!d) return fail(SOP_ERR_INVALID, "desc is NULL");
  const int nd = d->grid.ndim;
  if (nd != 1 && nd != 3) return fail(SOP_ERR_UNSUPPORTED, "ndim must be 1 or 3");
  for (int a = 0; a < nd; ++a) {
    if (d->grid.n[a] < 1) return fail(SOP_ERR_INVALID, "grid size must be positive");
    if (!(d->grid.hi[a] > d->grid.lo[a]) || !std::isfinite(d->grid.hi[a] - d->grid.lo[a]))
      return fail(SOP_ERR_INVALID, "grid requires lo < hi");
    if (!supported_length(nd, d->grid.n[a]))
      return fail(SOP_ERR_UNSUPPORTED, "unsupported grid length " + std::to_string(d->grid.n[a]));
  }
  if (nd == 3 && (d->grid.n[1] != d->grid.n[0] || d->grid.n[2] != d->grid.n[0]))
    return fail(SOP_ERR_UNSUPPORTED, "3D grids must be cubic");
  if (d->nsurf < 1 || (nd == 1 && d->nsurf > 2) || (nd == 3 && d->nsurf > 3))
    return fail(SOP_ERR_UNSUPPORTED, "nsurf must be 1..2 (1D) or 1..3 (3D)");
  if (!d->inv_mass || !d->vtable) return fail(SOP_ERR_INVALID, "inv_mass and vtable are required");
  for (int a = 0; a < nd; ++a)
    if (!std::isfinite(d->inv_mass[a]) || d->inv_mass[a] < 0)
      return fail(SOP_ERR_INVALID, "inv_mass must be finite and >= 0");
  if (!(d->dt != 0) || !std::isfinite(d->dt)) return fail(SOP_ERR_INVALID, "dt must be finite and nonzero");
  if (!(d->hbar > 0) || !std::isfinite(d->hbar)) return fail(SOP_ERR_INVALID, "hbar must be > 0");
  if (d->dtype != SOP_C128 && d->dtype != SOP_C64) return fail(SOP_ERR_INVALID, "bad dtype");
  if (d->nparams < 0 || d->nparams > sop::kMaxParams)
    return fail(SOP_ERR_INVALID, "nparams must be 0..8");
  if (d->nparams > 0 && !d->dvtables) return fail(SOP_ERR_INVALID, "dvtables required");
  return SOP_OK;
}

sop_status ensure_scratch(sop_plan* p) {
  if (!p->d_scratch) HIPTRY(dalloc(p, &p->d_scratch, (size_t)p->S * p->npts * p->csize));
  return SOP_OK;
}

}  // namespace

extern "C" {

int sop_abi_version(void) { return SOP_ABI_VERSION; }

const char* sop_status_string(sop_status s) {
  switch (s) {
    case SOP_OK: return "ok";
    case SOP_ERR_INVALID: return "invalid argument";
    case SOP_ERR_UNSUPPORTED: return "unsupported";
    case SOP_ERR_NOMEM: return "out of device memory";
    case SOP_ERR_HIP: return "HIP runtime error";
    case SOP_ERR_STATE: return "invalid state";
  }
  return "unknown status";
}

const char* sop_last_error(void) { return g_err.c_str(); }

int sop_supported_length(int ndim, int n) { return supported_length(ndim, n) ? 1 : 0; }

namespace {
sop_status write_sequence(const Sequence& s, int cap, double* a, double* b, double* a_unq,
                          double* b_unq, int* ia, int* ib, int* counts) {
  const int N = (int)s.a.size();
  if (cap < N) return fail(SOP_ERR_INVALID, "capacity smaller than the sequence length");
  for (int j = 0; j < N; ++j) {
    if (a) a[j] = s.a[j];
    if (b) b[j] = j < (int)s.b.size() ? s.b[j] : 0.0;
    if (ia) ia[j] = s.ia[j];
    if (ib) ib[j] = j < (int)s.ib.size() ? s.ib[j] : -1;
  }
  for (size_t u = 0; u < s.au.size(); ++u)
    if (a_unq) a_unq[u] = s.au[u];
  for (size_t u = 0; u < s.bu.size(); ++u)
    if (b_unq) b_unq[u] = s.bu[u];
  if (counts) {
    counts[0] = N;
    counts[1] = (int)s.au.size();
    counts[2] = (int)s.bu.size();
    counts[3] = s.M;
  }
  return SOP_OK;
}
}  // namespace

sop_status sop_scheme_sequence(sop_split split, sop_comp comp, int order, int cap, double* a,
                               double* b, double* a_unq, double* b_unq, int* ia, int* ib,
                               int* counts) {
  if (comp == SOP_COMP_CUSTOM)
    return fail(SOP_ERR_INVALID, "custom compositions go through sop_custom_sequence");
  Sequence s;
  const sop_status st = build_sequence(split, comp, order, 0, nullptr, s);
  if (st != SOP_OK) return st;
  return write_sequence(s, cap, a, b, a_unq, b_unq, ia, ib, counts);
}

sop_status sop_custom_sequence(sop_split split, int ngamma, const double* gamma, int cap,
                               double* a, double* b, double* a_unq, double* b_unq, int* ia,
                               int* ib, int* counts) {
  Sequence s;
  const sop_status st = build_sequence(split, SOP_COMP_CUSTOM, 2, ngamma, gamma, s);
  if (st != SOP_OK) return st;
  return write_sequence(s, cap, a, b, a_unq, b_unq, ia, ib, counts);
}

sop_status sop_plan_create(const sop_plan_desc* desc, void* hip_stream, sop_plan** out) {
  return sop_plan_create_with_allocator(desc, hip_stream, nullptr, out);
}

sop_status sop_plan_create_with_allocator(const sop_plan_desc* desc, void* hip_stream,
                                          const sop_allocator* allocator, sop_plan** out) {
  if (!out) return fail(SOP_ERR_INVALID, "out is NULL");
  if (allocator && (!allocator->alloc || !allocator->free))
    return fail(SOP_ERR_INVALID, "an allocator needs both alloc and free");
  sop_status st = validate(desc);
  if (st != SOP_OK) return st;
  sop_plan* p = new (std::nothrow) sop_plan();
  if (!p) return fail(SOP_ERR_NOMEM, "host allocation failed");
  if (allocator) p->hook = *allocator;
  p->home = (hipStream_t)hip_stream;
  struct Guard {
    sop_plan* p;
    bool keep = false;
    ~Guard() {
      if (!keep) free_plan(p);
    }
  } guard{p};

  st = build_sequence(desc->split, desc->comp, desc->order, desc->ngamma, desc->gamma, p->seq);
  if (st != SOP_OK) return st;
  p->ndim = desc->grid.ndim;
  p->S = desc->nsurf;
  p->npts = 1;
  p->dV = 1;
  for (int a = 0; a < p->ndim; ++a) {
    p->n[a] = desc->grid.n[a];
    p->lo[a] = desc->grid.lo[a];
    p->hi[a] = desc->grid.hi[a];
    p->dx[a] = (p->hi[a] - p->lo[a]) / p->n[a];
    p->inv_mass[a] = desc->inv_mass[a];
    p->npts *= p->n[a];
    p->dV *= p->dx[a];
  }
  p->dt = desc->dt;
  p->hbar = desc->hbar;
  p->dtype = desc->dtype;
  const bool f64 = desc->dtype == SOP_C128;
  p->csize = f64 ? 16 : 8;
  const int S = p->S, NE = S * (S + 1) / 2;
  hipStream_t stream = (hipStream_t)hip_stream;

  // coefficient sets: potential and kinetic
  const Sequence& q = p->seq;
  const std::vector<double>& vc = q.a_is_v ? q.au : q.bu;
  const std::vector<double>& tc = q.a_is_v ? q.bu : q.au;
  for (double c : vc) p->vtaus.push_back((double)((ld)c * (ld)p->dt / (ld)p->hbar));
  for (double c : tc) p->ttaus.push_back((double)((ld)c * (ld)p->dt));

  // step program
  std::vector<int> prog;
  const int nA = (int)q.a.size(), nB = (int)q.b.size();
  const int opA = q.a_is_v ? sop::OP_V : sop::OP_T, opB = q.a_is_v ? sop::OP_T : sop::OP_V;
  for (int j = 0; j < nA; ++j) {
    prog.push_back(sop::prog_entry(opA, q.ia[j]));
    if (j < nB) prog.push_back(sop::prog_entry(opB, q.ib[j]));
  }

  // device buffers
  const size_t vbytes = (size_t)NE * p->npts * sizeof(double);
  // 3D plans of two or three surfaces store the compact FP64 eigen form of
  // V (one table for every coefficient) instead of one exp(-i tau V) table
  // per unique coefficient; FP32 tables hold (rounded, residue) pairs
  const int rep = f64 ? 1 : 2;
  if (sop::eig_form(p->ndim, S)) {
    p->vbound = gershgorin_bound(desc->vtable, S, p->npts);
    for (int k = 0; k < desc->nparams; ++k)
      p->dvbound.push_back(gershgorin_bound(desc->dvtables + (size_t)k * NE * p->npts, S, p->npts));
    p->eig_form = phases_fit(p, p->vbound);
  }
  const size_t tbytes = p->eig_form ? (size_t)sop::eig_slots(S) * p->npts * 2 * sizeof(double)
                                    : vc.size() * NE * p->npts * p->csize * rep;
  const int nax = p->ndim == 1 ? 1 : 3;
  const size_t kbytes = tc.size() * nax * p->n[0] * p->csize * rep;
  const size_t wbytes = (size_t)nax * p->n[0] * p->csize * rep;
  if (dalloc(p, &p->d_vraw, vbytes) != hipSuccess || dalloc(p, &p->d_vexp, tbytes) != hipSuccess ||
      dalloc(p, &p->d_kin, kbytes) != hipSuccess || dalloc(p, &p->d_tw, wbytes) != hipSuccess ||
      dalloc(p, &p->d_prog, prog.size() * sizeof(int)) != hipSuccess ||
      dalloc(p, &p->d_prog1, 2 * sizeof(int)) != hipSuccess ||
      dalloc(p, &p->d_taus, (vc.size() + 1) * sizeof(double)) != hipSuccess ||
      dalloc(p, &p->d_part,
             (size_t)sop::kReduceBlocks * (S + 2 + sop::kMaxParams) * sizeof(double)) !=
          hipSuccess ||
      dalloc(p, &p->d_out, 8 * sizeof(double)) != hipSuccess) {
    (void)hipGetLastError();
    return fail(SOP_ERR_NOMEM, "device allocation failed for the plan tables");
  }
  p->table_bytes = tbytes + kbytes;

  // twiddles exp(-2 pi i k/n), one block per axis
  std::vector<ld> tw((size_t)nax * p->n[0] * 2);
  for (int a = 0; a < nax; ++a)
    for (int k = 0; k < p->n[a]; ++k) {
      const ld ang = -kTwoPi * (ld)k / (ld)p->n[a];
      tw[((size_t)a * p->n[0] + k) * 2] = std::cos(ang);
      tw[((size_t)a * p->n[0] + k) * 2 + 1] = std::sin(ang);
    }
  std::vector<char> twp = pack_split(tw, f64, p->n[0]);
  std::vector<char> kinp = pack_split(kinetic_factors(p, p->ttaus), f64, p->n[0]);
  const int prog1[2] = {sop::prog_entry(sop::OP_V, 0), sop::prog_entry(sop::OP_T, 0)};
  HIPTRY(hipMemcpyAsync(p->d_vraw, desc->vtable, vbytes, hipMemcpyHostToDevice, stream));
  HIPTRY(hipMemcpyAsync(p->d_tw, twp.data(), wbytes, hipMemcpyHostToDevice, stream));
  HIPTRY(hipMemcpyAsync(p->d_kin, kinp.data(), kbytes, hipMemcpyHostToDevice, stream));
  HIPTRY(hipMemcpyAsync(p->d_prog, prog.data(), prog.size() * sizeof(int), hipMemcpyHostToDevice,
                        stream));
  HIPTRY(hipMemcpyAsync(p->d_prog1, prog1, sizeof(prog1), hipMemcpyHostToDevice, stream));
  HIPTRY(hipMemcpyAsync(p->d_taus, p->vtaus.data(), p->vtaus.size() * sizeof(double),
                        hipMemcpyHostToDevice, stream));

  DevView& d = p->dv;
  d.ndim = p->ndim;
  for (int a = 0; a < 3; ++a) d.n[a] = a < p->ndim ? p->n[a] : 1;
  d.S = S;
  d.npts = p->npts;
  d.f64 = f64;
  d.stream = stream;
  d.vexp = p->d_vexp;
  d.kin = p->d_kin;
  d.kin_stride = p->n[0] * rep;
  for (int a = 0; a < 3; ++a)
    d.tw[a] = (const char*)p->d_tw + (size_t)(a < nax ? a : 0) * p->n[0] * p->csize * rep;
  d.prog = p->d_prog;
  d.nact = (int)prog.size();
  d.hprog = prog;
  // the plane pass has one workgroup per plane and surface: it wins on small
  // grids, where the separate passes cannot fill the chip either, and loses
  // to them on 128^3 (one 139 KB workgroup per compute unit)
  d.plane = p->ndim == 3 && p->n[0] <= 64;

  p->tile = p->ndim == 3 ? sop::k3d_table_tile(p->n[0], f64) : 0;
  d.vtaus = p->d_taus;
  d.eig = p->eig_form;
  HIPTRY(form_tables(p));
  if (p->ndim == 3) {
    p->graphs = new (std::nothrow) sop::GraphCache();
    if (!p->graphs) return fail(SOP_ERR_NOMEM, "host allocation failed");
    HIPTRY(hipStreamCreateWithFlags(&p->graphs->capture, hipStreamNonBlocking));
    d.graphs = p->graphs;
  }
  p->nparams = desc->nparams;
  if (p->nparams > 0) {
    const size_t dvb = (size_t)p->nparams * vbytes;
    if (dalloc(p, &p->d_vbase, vbytes) != hipSuccess || dalloc(p, &p->d_dv, dvb) != hipSuccess ||
        dalloc(p, &p->d_theta, sop::kMaxParams * sizeof(double)) != hipSuccess ||
        dalloc(p, &p->d_w, 8 * sizeof(double)) != hipSuccess) {
      (void)hipGetLastError();
      return fail(SOP_ERR_NOMEM, "device allocation failed for the parameter tables");
    }
    HIPTRY(hipMemcpyAsync(p->d_vbase, p->d_vraw, vbytes, hipMemcpyDeviceToDevice, stream));
    HIPTRY(hipMemcpyAsync(p->d_dv, desc->dvtables, dvb, hipMemcpyHostToDevice, stream));
    p->theta.assign(p->nparams, 0.0);  // the V-table is V at theta = 0
    HIPTRY(hipMemcpyAsync(p->d_theta, p->theta.data(), p->nparams * sizeof(double),
                          hipMemcpyHostToDevice, stream));
    if (p->ndim == 3 && f64 && sop::k3d_adjoint_supported(p->n[0], S, f64)) {
      const int nslots = S >= 2 ? sop::eig_slots(S) : NE;  // compact eigen form for S >= 2
      if (dalloc(p, &p->d_eig, (size_t)nslots * p->npts * sizeof(double) * 2) != hipSuccess) {
        (void)hipGetLastError();
        return fail(SOP_ERR_NOMEM, "device allocation failed for the eigen table");
      }
      HIPTRY(sop::form_eig(d, p->d_vraw, p->tile, p->d_eig));
    }
  }
  HIPTRY(hipStreamSynchronize(stream));
  guard.keep = true;
  *out = p;
  return SOP_OK;
}

sop_status sop_plan_destroy(sop_plan* plan) {
  if (plan) {
    (void)hipStreamSynchronize(plan->dv.stream);
    free_plan(plan);
  }
  return SOP_OK;
}

sop_status sop_plan_info_get(const sop_plan* p, sop_plan_info* out) {
  if (!p || !out) return fail(SOP_ERR_INVALID, "NULL argument");
  sop_plan_info i;
  std::memset(&i, 0, sizeof(i));
  i.M = p->seq.M;
  i.n_a = (int)p->seq.a.size();
  i.n_b = (int)p->seq.b.size();
  i.n_a_unq = (int)p->seq.au.size();
  i.n_b_unq = (int)p->seq.bu.size();
  i.n_v_tables = p->eig_form ? 1 : (int)p->vtaus.size();
  i.n_t_tables = (int)p->ttaus.size();
  i.npts = p->npts;
  i.table_bytes = p->table_bytes;
  i.scratch_bytes = (size_t)p->S * p->npts * p->csize;
  *out = i;
  return SOP_OK;
}

sop_status sop_plan_set_stream(sop_plan* p, void* hip_stream) {
  if (!p) return fail(SOP_ERR_INVALID, "plan is NULL");
  p->dv.stream = (hipStream_t)hip_stream;
  return SOP_OK;
}

sop_status sop_propagate(sop_plan* p, void* psi, int64_t nsteps, int direction) {
  if (!p || !psi) return fail(SOP_ERR_INVALID, "NULL argument");
  if (nsteps < 0) return fail(SOP_ERR_INVALID, "nsteps must be >= 0");
  if (direction != 1 && direction != -1) return fail(SOP_ERR_INVALID, "direction must be +1 or -1");
  if (nsteps == 0) return SOP_OK;
  const int conj = direction < 0 ? 1 : 0;
  if (p->graphs && p->graphs->execs.size() > 48) {
    HIPTRY(hipStreamSynchronize(p->dv.stream));
    p->graphs->clear();
  }
  if (p->ndim == 1)
    HIPTRY(sop::k1d_propagate(p->dv, psi, nsteps, conj));
  else
    HIPTRY(sop::k3d_propagate(p->dv, psi, nsteps, conj));
  return SOP_OK;
}

sop_status sop_propagate_many(sop_plan* p, void* psi, int count, int64_t nsteps, int direction) {
  if (!p || !psi) return fail(SOP_ERR_INVALID, "NULL argument");
  if (count < 1 || count > 65535) return fail(SOP_ERR_INVALID, "count must be 1..65535");
  if (nsteps < 0) return fail(SOP_ERR_INVALID, "nsteps must be >= 0");
  if (direction != 1 && direction != -1) return fail(SOP_ERR_INVALID, "direction must be +1 or -1");
  if (nsteps == 0) return SOP_OK;
  const int conj = direction < 0 ? 1 : 0;
  if (p->ndim == 1) {
    HIPTRY(sop::k1d_propagate(p->dv, psi, nsteps, conj, count));
  } else {
    sop::DevView d = p->dv;
    d.count = count;
    HIPTRY(sop::k3d_propagate(d, psi, nsteps, conj));
  }
  return SOP_OK;
}

sop_status sop_observables(sop_plan* p, const void* psi, double* out) {
  if (!p || !psi || !out) return fail(SOP_ERR_INVALID, "NULL argument");
  sop_status st = ensure_scratch(p);
  if (st != SOP_OK) return st;
  const size_t bytes = (size_t)p->S * p->npts * p->csize;
  HIPTRY(hipMemcpyAsync(p->d_scratch, psi, bytes, hipMemcpyDeviceToDevice, p->dv.stream));
  if (p->ndim == 1)
    HIPTRY(sop::k1d_fft_forward(p->dv, p->d_scratch));
  else
    HIPTRY(sop::k3d_fft_forward(p->dv, p->d_scratch));
  HIPTRY(sop::obs_reduce(p->dv, psi, p->d_scratch, p->d_vraw, p->inv_mass, p->dx, p->hbar,
                         p->d_part, p->d_out));
  double raw[8];
  HIPTRY(hipMemcpyAsync(raw, p->d_out, (p->S + 2) * sizeof(double), hipMemcpyDeviceToHost,
                        p->dv.stream));
  HIPTRY(hipStreamSynchronize(p->dv.stream));
  const int S = p->S;
  double norm = 0;
  for (int s = 0; s < S; ++s) norm += raw[s] * p->dV;
  const double ev = raw[S] * p->dV;
  const double et = raw[S + 1] * p->dV / (double)p->npts;
  out[0] = norm;
  out[1] = et + ev;
  for (int s = 0; s < S; ++s) out[2 + s] = raw[s] * p->dV;
  out[2 + S] = et;
  out[3 + S] = ev;
  return SOP_OK;
}

sop_status sop_overlap(sop_plan* p, const void* psi, const void* phi, double* out) {
  if (!p || !psi || !phi || !out) return fail(SOP_ERR_INVALID, "NULL argument");
  HIPTRY(sop::overlap_reduce(p->dv, psi, phi, p->d_part, p->d_out));
  double raw[2];
  HIPTRY(hipMemcpyAsync(raw, p->d_out, 2 * sizeof(double), hipMemcpyDeviceToHost, p->dv.stream));
  HIPTRY(hipStreamSynchronize(p->dv.stream));
  out[0] = raw[0] * p->dV;
  out[1] = raw[1] * p->dV;
  return SOP_OK;
}

sop_status sop_distance(sop_plan* p, const void* psi, const void* phi, double* out) {
  if (!p || !psi || !phi || !out) return fail(SOP_ERR_INVALID, "NULL argument");
  HIPTRY(sop::distance_reduce(p->dv, psi, phi, p->d_part, p->d_out));
  double raw[2];
  HIPTRY(hipMemcpyAsync(raw, p->d_out, 2 * sizeof(double), hipMemcpyDeviceToHost, p->dv.stream));
  HIPTRY(hipStreamSynchronize(p->dv.stream));
  out[0] = std::sqrt(raw[0] * p->dV);
  out[1] = raw[1] > 0.0 ? std::sqrt(raw[0] / raw[1]) : 0.0;
  return SOP_OK;
}

}  // extern "C"

namespace {

// Device workspace of the trapezoidal rule.  1D: count S N complex
// residuals, the per-state statistics (three int64 each) and the stage
// coefficients.  3D (one state at a time): six state-sized vectors (r, p,
// A p and the three one-axis kinetic terms), the reduction partials and
// sums, and the factor block T_d(k)/n_d of the three axes.
struct TrapLayout {
  size_t vec = 0, sbytes = 0, need = 0;
  int nst = 0;
  bool three_d = false;
  size_t one = 0;  // 3D: bytes of one state-sized vector
};

sop_status trap_check(const sop_plan* p, const void* psi, int count, int64_t nsteps, double tol,
                      int max_iter, TrapLayout* lay) {
  if (!p || !psi) return fail(SOP_ERR_INVALID, "NULL argument");
  if (count < 1 || count > 65535) return fail(SOP_ERR_INVALID, "count must be 1..65535");
  if (nsteps < 0) return fail(SOP_ERR_INVALID, "nsteps must be >= 0");
  if (!(tol > 0) || !(tol < 1)) return fail(SOP_ERR_INVALID, "tol must be in (0, 1)");
  if (max_iter < 1) return fail(SOP_ERR_INVALID, "max_iter must be >= 1");
  if (p->dtype != SOP_C128 ||
      !(p->ndim == 3 || (p->ndim == 1 && sop::k1d_trap_supported(p->n[0], p->S))))
    return fail(SOP_ERR_UNSUPPORTED,
                "the trapezoidal rule runs on SOP_C128 plans: 1D of 512..8192 points, or 3D");
  if (p->seq.g.empty())
    return fail(SOP_ERR_INVALID, "the plan's splitting has no composition (VT/TV)");
  lay->nst = (int)p->seq.g.size();
  if (p->ndim == 3) {
    lay->three_d = true;
    lay->one = ((size_t)p->S * p->npts * sizeof(double2) + 255) / 256 * 256;
    lay->need = 6 * lay->one + ((size_t)sop::kT3Partials + sop::kT3Status) * sizeof(double) +
                (size_t)3 * p->n[0] * sizeof(double2);
    return SOP_OK;
  }
  lay->vec = (size_t)count * p->S * p->n[0] * sizeof(double2);
  lay->sbytes = ((size_t)count * 3 * sizeof(long long) + 255) / 256 * 256;
  lay->need = lay->vec + lay->sbytes + (size_t)lay->nst * sizeof(double);
  return SOP_OK;
}

// The trapezoidal rule on a 3D plan: for every state and stage, conjugate
// orthogonal CG on (1 + i tau H) x = (1 - i tau H) psi started from x = psi,
// H u = sum_d F_d^-1 T_d(k) F_d u + V u, the kinetic terms computed by the
// propagator's one-axis passes reading u.  The host enqueues the
// iterations and reads the device's status block every few of them (the
// scalars of the method stay on the device); every device reduction is in
// a fixed order.  Synchronises.
sop_status trap3d_run(sop_plan* p, void* psi, int count, int64_t nsteps, double tol,
                      int max_iter, char* base, const TrapLayout& lay, bool allow_graphs,
                      int64_t* iterations) {
  const DevView& d = p->dv;
  hipStream_t st = d.stream;
  const int S = p->S, n = p->n[0];
  const int64_t npts = p->npts, nall = (int64_t)S * npts;
  const size_t one = lay.one;
  sop::Trap3Bufs b;
  b.r = base;
  b.p = base + one;
  b.ap = base + 2 * one;
  b.qz = base + 3 * one;
  b.qy = base + 4 * one;
  b.qx = base + 5 * one;
  b.partials = (double*)(base + 6 * one);
  b.sums = b.partials + (size_t)sop::kT3Partials;
  double2* hfac = (double2*)(b.sums + sop::kT3Status);
  // T_d(k) / n_d on the signed frequencies of each axis (the 1/n_d of the
  // unnormalised inverse transform folded in, as in the kinetic factors)
  std::vector<double2> hf((size_t)3 * n);
  for (int a = 0; a < 3; ++a)
    for (int k = 0; k < n; ++k) {
      const int kk = k < n / 2 ? k : k - n;
      const ld kap = kTwoPi * (ld)kk / ((ld)p->n[a] * (ld)p->dx[a]);
      hf[(size_t)a * n + k] = {(double)((ld)p->hbar * p->hbar * kap * kap *
                                        (ld)p->inv_mass[a] / 2.0L / (ld)p->n[a]),
                               0.0};
    }
  HIPTRY(hipMemcpyAsync(hfac, hf.data(), hf.size() * sizeof(double2), hipMemcpyHostToDevice, st));
  DevView dh = d;
  dh.kin = hfac;
  dh.kin_stride = n;
  dh.count = 1;
  dh.graphs = nullptr;
  dh.timer = nullptr;
  const size_t bytes = (size_t)nall * sizeof(double2);
  // the three one-axis kinetic terms of H u, on stream s (each pass reads u
  // and writes its own term)
  auto kinetic = [&](const void* u, hipStream_t s) -> sop_status {
    void* q[3] = {b.qz, b.qy, b.qx};
    dh.stream = s;
    for (int a = 0; a < 3; ++a) HIPTRY(sop::k3d_axis_kinetic(dh, q[a], a, u));
    return SOP_OK;
  };
  // kBlock iterations of stage coefficient tau, on stream s
  constexpr int kBlock = 4;
  static_assert(kBlock % 2 == 0, "iteration parity per block");
  auto block = [&](double tau, hipStream_t s) -> sop_status {
    sop_status r;
    for (int i = 0; i < kBlock; ++i) {  // kBlock is even: the parity restarts
      if ((r = kinetic(b.p, s)) != SOP_OK) return r;
      HIPTRY(sop::t3_ap(b, S, p->d_vraw, npts, tau, s));
      HIPTRY(sop::t3_update(b, S, npts, i & 1, s));
      HIPTRY(sop::t3_pupdate(b, S, npts, i & 1, s));
    }
    return SOP_OK;
  };
  // the block as a graph captured once per (state, workspace, tau): its
  // launches then cost one graph launch (none for the allocation-free call,
  // whose contract rules out instantiating graphs)
  const bool use_graph = allow_graphs && p->use_graphs && p->graphs && p->graphs->capture;
  auto run_block = [&](double tau) -> sop_status {
    if (!use_graph) return block(tau, st);
    uint64_t tb;
    std::memcpy(&tb, &tau, sizeof(tb));
    const sop_plan::T3Key key{b.x, base, tb};
    auto it = p->t3graphs.find(key);
    if (it == p->t3graphs.end()) {
      if (p->t3graphs.size() >= 64) {
        for (auto& kv : p->t3graphs) (void)hipGraphExecDestroy(kv.second);
        p->t3graphs.clear();
      }
      hipStream_t cs = p->graphs->capture;
      HIPTRY(hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal));
      const sop_status bs = block(tau, cs);
      hipGraph_t g = nullptr;
      const hipError_t ce = hipStreamEndCapture(cs, &g);
      dh.stream = st;
      if (bs != SOP_OK) {
        if (g) (void)hipGraphDestroy(g);
        return bs;
      }
      HIPTRY(ce);
      hipGraphExec_t x = nullptr;
      const hipError_t ie = hipGraphInstantiate(&x, g, nullptr, nullptr, 0);
      (void)hipGraphDestroy(g);
      HIPTRY(ie);
      it = p->t3graphs.emplace(key, x).first;
    }
    HIPTRY(hipGraphLaunch(it->second, st));
    return SOP_OK;
  };
  double stat[sop::kT3Status];
  auto read = [&]() -> sop_status {
    HIPTRY(hipMemcpyAsync(stat, b.sums, sizeof(stat), hipMemcpyDeviceToHost, st));
    HIPTRY(hipStreamSynchronize(st));
    return SOP_OK;
  };
  // iterations of the last solve of each stage: the status is read after
  // each block once that many are near (the status freezes the iterate once
  // the test holds, so iterations past it change nothing)
  std::vector<int> expect(lay.nst, 0);
  const double tol2 = tol * tol;
  int64_t total = 0, failed = 0;
  sop_status sts;
  for (int c = 0; c < count; ++c) {
    b.x = (char*)psi + (size_t)c * bytes;
    for (int64_t step = 0; step < nsteps; ++step)
      for (int j = 0; j < lay.nst; ++j) {
        const double tau = (double)((ld)p->seq.g[j] * (ld)p->dt / (2 * (ld)p->hbar));
        if ((sts = kinetic(b.x, st)) != SOP_OK) return sts;
        HIPTRY(sop::t3_init(b, S, p->d_vraw, npts, tau, tol2, max_iter, st));
        int launched = 0;
        bool stop = false;
        while (!stop && launched < max_iter) {
          if ((sts = run_block(tau)) != SOP_OK) return sts;
          launched += kBlock;
          if (launched + kBlock > expect[j] || launched >= max_iter) {
            if ((sts = read()) != SOP_OK) return sts;
            stop = stat[sop::T3_STOP] != 0.0;
          }
        }
        const int it = (int)stat[sop::T3_ITER];
        expect[j] = it;
        total += it;
        const bool met = stat[sop::T3_RR] <= stat[sop::T3_TOL2] * stat[sop::T3_BB];
        if (!stop || !met || stat[sop::T3_FAIL] != 0.0) ++failed;
      }
  }
  HIPTRY(hipStreamSynchronize(st));
  if (iterations) *iterations = total;
  if (failed > 0)
    return fail(SOP_ERR_STATE, std::to_string(failed) + " of the linear solves did not reach tol in " +
                                   std::to_string(max_iter) + " iterations");
  return SOP_OK;
}

// Runs the trapezoidal-rule compositions with the workspace at `base`
// (device, lay.need bytes; nothing in it needs clearing: every element is
// written before it is read).  Synchronises the plan's stream.
sop_status trap_run(sop_plan* p, void* psi, int count, int64_t nsteps, double tol, int max_iter,
                    char* base, const TrapLayout& lay, bool allow_graphs, int64_t* iterations) {
  if (lay.three_d)
    return trap3d_run(p, psi, count, nsteps, tol, max_iter, base, lay, allow_graphs, iterations);
  const int nst = lay.nst;
  std::vector<double> taus(nst);
  for (int j = 0; j < nst; ++j) taus[j] = (double)((ld)p->seq.g[j] * (ld)p->dt / (2 * (ld)p->hbar));
  const DevView& d = p->dv;
  HIPTRY(hipMemcpyAsync(base + lay.vec + lay.sbytes, taus.data(), nst * sizeof(double),
                        hipMemcpyHostToDevice, d.stream));
  sop::TrapArgs g;
  g.psi = psi;
  g.rbuf = base;
  g.vraw = p->d_vraw;
  g.taus = (const double*)(base + lay.vec + lay.sbytes);
  g.nst = nst;
  g.nsteps = nsteps;
  const ld L = (ld)p->hi[0] - (ld)p->lo[0];
  const ld kap = kTwoPi / L;
  g.tk = (double)((ld)p->hbar * p->hbar * p->inv_mass[0] * kap * kap / 2);
  g.tol2 = tol * tol;
  g.maxit = max_iter;
  g.stats = (long long*)(base + lay.vec);
  g.count = count;
  {
    sop::TimedLaunch tl(d, sop::KIND_1D, 0.0);
    HIPTRY(sop::k1d_trapezoid(d, g));
  }
  std::vector<long long> st((size_t)count * 3);
  HIPTRY(hipMemcpyAsync(st.data(), g.stats, st.size() * sizeof(long long), hipMemcpyDeviceToHost,
                        d.stream));
  HIPTRY(hipStreamSynchronize(d.stream));
  int64_t total = 0, failed = 0;
  for (int c = 0; c < count; ++c) {
    total += st[3 * c];
    failed += st[3 * c + 1];
  }
  if (iterations) *iterations = total;
  if (failed > 0)
    return fail(SOP_ERR_STATE, std::to_string(failed) + " of the linear solves did not reach tol in " +
                                   std::to_string(max_iter) + " iterations");
  return SOP_OK;
}

}  // namespace

extern "C" {

sop_status sop_propagate_trapezoid(sop_plan* p, void* psi, int count, int64_t nsteps, double tol,
                                   int max_iter, int64_t* iterations) {
  TrapLayout lay;
  const sop_status st = trap_check(p, psi, count, nsteps, tol, max_iter, &lay);
  if (st != SOP_OK) return st;
  if (lay.need > p->trap_bytes) {
    if (p->d_trap) {
      HIPTRY(hipStreamSynchronize(p->dv.stream));
      if (p->hook.free)
        p->hook.free(p->hook.ctx, p->d_trap, (void*)p->home);
      else
        HIPTRY(hipFree(p->d_trap));
      p->d_trap = nullptr;
      p->trap_bytes = 0;
    }
    if (dalloc(p, &p->d_trap, lay.need) != hipSuccess)
      return fail(SOP_ERR_NOMEM, "trapezoid workspace");
    p->trap_bytes = lay.need;
  }
  return trap_run(p, psi, count, nsteps, tol, max_iter, (char*)p->d_trap, lay, true, iterations);
}

sop_status sop_propagate_trapezoid_noalloc(sop_plan* p, void* psi, int count, int64_t nsteps,
                                           double tol, int max_iter, int64_t* iterations) {
  TrapLayout lay;
  const sop_status st = trap_check(p, psi, count, nsteps, tol, max_iter, &lay);
  if (st != SOP_OK) return st;
  const size_t cap = sop::trap_scratch_bytes();
  if (lay.need > cap)
    return fail(SOP_ERR_INVALID,
                "count * nsurf * N complex residuals plus statistics and coefficients need " +
                    std::to_string(lay.need) + " bytes, more than the static scratch of " +
                    std::to_string(cap) + " bytes");
  void* base = nullptr;
  HIPTRY(sop::trap_scratch(p->dv.stream, &base));
  return trap_run(p, psi, count, nsteps, tol, max_iter, (char*)base, lay, false, iterations);
}

sop_status sop_interpolate(const sop_plan* src, const void* psi_src, sop_plan* dst,
                           void* psi_dst) {
  if (!src || !dst || !psi_src || !psi_dst) return fail(SOP_ERR_INVALID, "NULL argument");
  if (psi_src == psi_dst) return fail(SOP_ERR_INVALID, "psi_src and psi_dst must differ");
  if (src->ndim != dst->ndim || src->S != dst->S)
    return fail(SOP_ERR_INVALID, "plans differ in ndim or nsurf");
  if (src->dtype != SOP_C128 || dst->dtype != SOP_C128)
    return fail(SOP_ERR_UNSUPPORTED, "interpolation is implemented for SOP_C128 plans");
  const int nax = src->ndim;
  for (int a = 0; a < nax; ++a)
    if (dst->n[a] > 65535) return fail(SOP_ERR_UNSUPPORTED, "destination axis too long");
  const int S = src->S;
  // axis a of the arrays: 0 slowest; 1D grids use axis 0 only
  const long long ns[3] = {src->n[0], nax == 3 ? src->n[1] : 1, nax == 3 ? src->n[2] : 1};
  const long long nd[3] = {dst->n[0], nax == 3 ? dst->n[1] : 1, nax == 3 ? dst->n[2] : 1};
  // workspace: the axis matrices, then (3D) the state after z and after y
  size_t wel = 0;
  for (int a = 0; a < nax; ++a) wel += (size_t)nd[a] * ns[a];
  const size_t t1 = nax == 3 ? (size_t)S * ns[0] * ns[1] * nd[2] : 0;
  const size_t t2 = nax == 3 ? (size_t)S * ns[0] * nd[1] * nd[2] : 0;
  const size_t need = (wel + t1 + t2) * sizeof(double2);
  if (need > dst->iws_bytes) {
    if (dst->d_iws) {
      HIPTRY(hipStreamSynchronize(dst->dv.stream));
      if (dst->hook.free)
        dst->hook.free(dst->hook.ctx, dst->d_iws, (void*)dst->home);
      else
        HIPTRY(hipFree(dst->d_iws));
      dst->d_iws = nullptr;
      dst->iws_bytes = 0;
    }
    dst->iws_valid = false;
    if (dalloc(dst, &dst->d_iws, need) != hipSuccess)
      return fail(SOP_ERR_NOMEM, "interpolation workspace");
    dst->iws_bytes = need;
  }
  // the axis matrices depend only on the two grids: formed again only when
  // the source grid differs from the last call's
  double key[9];
  for (int a = 0; a < 3; ++a) {
    key[3 * a] = (double)ns[a];
    key[3 * a + 1] = a < nax ? src->lo[a] : 0.0;
    key[3 * a + 2] = a < nax ? src->hi[a] : 0.0;
  }
  const bool reuse = dst->iws_valid && std::equal(key, key + 9, dst->iws_key);
  double2* W[3];
  double2* w = (double2*)dst->d_iws;
  for (int a = 0; a < nax; ++a) {
    W[a] = w;
    w += (size_t)nd[a] * ns[a];
  }
  double2* T1 = w;
  double2* T2 = w + t1;
  const DevView& d = dst->dv;
  if (!reuse) {
    dst->iws_valid = false;
    sop::TimedLaunch tl(d, sop::KIND_OTHER, (double)wel * sizeof(double2));
    for (int a = 0; a < nax; ++a)
      HIPTRY(sop::interp_weights(d.stream, W[a], (int)ns[a], src->lo[a], src->hi[a],
                                 (int)nd[a], dst->lo[a], dst->hi[a]));
    std::copy(key, key + 9, dst->iws_key);
    dst->iws_valid = true;
  }
  auto flops = [](const sop::CgemmArgs& g, int batch) {
    return 8.0 * g.M * (double)g.N * g.K * batch;
  };
  // Host check, before every launch, that the product's last elements lie
  // inside the buffers it reads and writes.
  auto fits = [](const sop::CgemmArgs& g, int batch, size_t na, size_t nb, size_t nc) {
    const long long b = batch - 1, m = g.M - 1, n = g.N - 1, k = g.K - 1;
    return (size_t)(b * g.bsa + m * g.sai + k * g.sak) < na &&
           (size_t)(b * g.bsb + k * g.sbk + n * g.sbj) < nb &&
           (size_t)(b * g.bsc + m * g.sci + n * g.scj) < nc;
  };
  const size_t nsrc = (size_t)S * ns[0] * ns[1] * ns[2];
  const size_t ndst = (size_t)S * nd[0] * nd[1] * nd[2];
  const int zax = nax - 1;  // the contiguous axis
  {  // along z: rows of the source times W_z^T
    sop::CgemmArgs g;
    g.A = (const double2*)psi_src;
    g.M = (int)(S * (nax == 3 ? ns[0] * ns[1] : 1));  // every line along z
    g.K = (int)ns[zax];
    g.N = (int)nd[zax];
    g.sai = g.K;
    g.sak = 1;
    g.B = W[zax];
    g.sbk = 1;
    g.sbj = g.K;
    g.C = nax == 3 ? T1 : (double2*)psi_dst;
    g.sci = g.N;
    g.scj = 1;
    if (!fits(g, 1, nsrc, (size_t)nd[zax] * ns[zax], nax == 3 ? t1 : ndst))
      return fail(SOP_ERR_INVALID, "interpolation: internal size check failed (z)");
    sop::TimedLaunch tl(d, sop::KIND_INTERP, flops(g, 1));
    HIPTRY(sop::cgemm(d.stream, g, 1));
  }
  if (nax == 3) {
    {  // along y: W_y times each (y, z) slab
      sop::CgemmArgs g;
      g.A = W[1];
      g.M = (int)nd[1];
      g.K = (int)ns[1];
      g.N = (int)nd[2];
      g.sai = g.K;
      g.sak = 1;
      g.B = T1;
      g.sbk = nd[2];
      g.sbj = 1;
      g.bsb = ns[1] * nd[2];
      g.C = T2;
      g.sci = nd[2];
      g.scj = 1;
      g.bsc = nd[1] * nd[2];
      const int batch = (int)(S * ns[0]);
      if (!fits(g, batch, (size_t)nd[1] * ns[1], t1, t2))
        return fail(SOP_ERR_INVALID, "interpolation: internal size check failed (y)");
      sop::TimedLaunch tl(d, sop::KIND_INTERP, flops(g, batch));
      HIPTRY(sop::cgemm(d.stream, g, batch));
    }
    {  // along x: W_x times each surface's (x, yz) matrix
      sop::CgemmArgs g;
      g.A = W[0];
      g.M = (int)nd[0];
      g.K = (int)ns[0];
      g.N = (int)(nd[1] * nd[2]);
      g.sai = g.K;
      g.sak = 1;
      g.B = T2;
      g.sbk = nd[1] * nd[2];
      g.sbj = 1;
      g.bsb = ns[0] * nd[1] * nd[2];
      g.C = (double2*)psi_dst;
      g.sci = nd[1] * nd[2];
      g.scj = 1;
      g.bsc = nd[0] * nd[1] * nd[2];
      if (!fits(g, S, (size_t)nd[0] * ns[0], t2, ndst))
        return fail(SOP_ERR_INVALID, "interpolation: internal size check failed (x)");
      sop::TimedLaunch tl(d, sop::KIND_INTERP, flops(g, S));
      HIPTRY(sop::cgemm(d.stream, g, S));
    }
  }
  return SOP_OK;
}

sop_status sop_apply_action(sop_plan* p, void* psi, int op, double coef) {
  if (!p || !psi) return fail(SOP_ERR_INVALID, "NULL argument");
  if (op != 0 && op != 1) return fail(SOP_ERR_INVALID, "op must be 0 (V) or 1 (T)");
  if (!std::isfinite(coef)) return fail(SOP_ERR_INVALID, "coef must be finite");
  DevView d = p->dv;
  if (op == 0) {
    const int NE = p->S * (p->S + 1) / 2;
    const double tau = (double)((ld)coef * (ld)p->dt / (ld)p->hbar);
    HIPTRY(hipMemcpyAsync(p->d_taus + p->vtaus.size(), &tau, sizeof(double),
                          hipMemcpyHostToDevice, d.stream));
    if (p->eig_form && std::fabs(tau) * p->vbound <= sop::kPhaseMax) {
      // the eigen form serves any tau within range: index the spare slot
      d.hprog = {sop::prog_entry(sop::OP_V, (int)p->vtaus.size())};
    } else {
      d.eig = false;
      if (!p->d_atab)
        HIPTRY(dalloc(p, &p->d_atab, (size_t)NE * p->npts * p->csize * (d.f64 ? 1 : 2)));
      HIPTRY(sop::form_vexp(d, p->d_vraw, p->d_taus + p->vtaus.size(), 1, p->tile, p->d_atab));
      d.vexp = p->d_atab;
      d.prog = p->d_prog1;
      d.hprog = {sop::prog_entry(sop::OP_V, 0)};
    }
  } else {
    const int nax = p->ndim == 1 ? 1 : 3;
    const size_t kb = (size_t)nax * p->n[0] * p->csize * (d.f64 ? 1 : 2);
    if (!p->d_akin) HIPTRY(dalloc(p, &p->d_akin, kb));
    std::vector<char> kp =
        pack_split(kinetic_factors(p, {(double)((ld)coef * (ld)p->dt)}), d.f64, p->n[0]);
    HIPTRY(hipMemcpyAsync(p->d_akin, kp.data(), kb, hipMemcpyHostToDevice, d.stream));
    d.kin = p->d_akin;
    d.prog = p->d_prog1 + 1;
    d.hprog = {sop::prog_entry(sop::OP_T, 0)};
  }
  d.nact = 1;
  if (p->ndim == 1)
    HIPTRY(sop::k1d_propagate(d, psi, 1, 0));
  else
    HIPTRY(sop::k3d_propagate(d, psi, 1, 0));
  // the host staging buffers above must outlive the copies
  HIPTRY(hipStreamSynchronize(d.stream));
  return SOP_OK;
}

sop_status sop_plan_set_params(sop_plan* p, const double* theta) {
  if (!p || !theta) return fail(SOP_ERR_INVALID, "NULL argument");
  if (p->nparams == 0) return fail(SOP_ERR_STATE, "plan has no parameters");
  for (int k = 0; k < p->nparams; ++k)
    if (!std::isfinite(theta[k])) return fail(SOP_ERR_INVALID, "theta must be finite");
  if (p->eig_form && !phases_fit(p, param_bound(p, p->vbound, theta)))
    return fail(SOP_ERR_UNSUPPORTED,
                "these parameters take the phases tau*lambda beyond the eigen form's range");
  hipStream_t st = p->dv.stream;
  HIPTRY(hipMemcpyAsync(p->d_theta, theta, p->nparams * sizeof(double), hipMemcpyHostToDevice, st));
  HIPTRY(sop::set_vparams(p->dv, p->d_vraw, p->d_vbase, p->d_dv, p->d_theta, p->nparams));
  HIPTRY(form_tables(p));
  if (p->d_eig) HIPTRY(sop::form_eig(p->dv, p->d_vraw, p->tile, p->d_eig));
  HIPTRY(hipStreamSynchronize(st));
  p->theta.assign(theta, theta + p->nparams);
  return SOP_OK;
}

sop_status sop_action_times(const sop_plan* p, double* c, int cap, int* count) {
  if (!p || !count) return fail(SOP_ERR_INVALID, "NULL argument");
  // the kinetic actions advance time; potential actions happen at an instant
  std::vector<double> t;
  double elapsed = 0.0;
  for (int code : p->dv.hprog) {
    if ((code >> 16) == sop::OP_V)
      t.push_back(elapsed);
    else
      elapsed += p->ttaus[code & 0xffff] / p->dt;
  }
  if (c && cap < (int)t.size()) return fail(SOP_ERR_INVALID, "cap is smaller than the count");
  if (c) std::copy(t.begin(), t.end(), c);
  *count = (int)t.size();
  return SOP_OK;
}

sop_status sop_propagate_driven(sop_plan* p, void* psi, int64_t nsteps, const double* drive) {
  if (!p || !psi) return fail(SOP_ERR_INVALID, "NULL argument");
  if (nsteps < 0) return fail(SOP_ERR_INVALID, "nsteps must be >= 0");
  if (p->nparams != 1)
    return fail(SOP_ERR_STATE, "a driven plan has exactly one parameter table (the drive's D)");
  int nv = 0;
  for (int code : p->dv.hprog) nv += (code >> 16) == sop::OP_V;
  const size_t ns = (size_t)nsteps * (size_t)nv;
  if (nsteps == 0) return SOP_OK;
  if (!drive) return fail(SOP_ERR_INVALID, "drive is NULL");
  double smax = 0.0;
  for (size_t i = 0; i < ns; ++i) {
    if (!std::isfinite(drive[i])) return fail(SOP_ERR_INVALID, "drive must be finite");
    smax = std::max(smax, std::fabs(drive[i]));
  }
  if (p->eig_form && !phases_fit(p, p->vbound + smax * p->dvbound[0]))
    return fail(SOP_ERR_UNSUPPORTED,
                "the drive takes the phases tau*lambda beyond the eigen form's range");
  hipStream_t st = p->dv.stream;
  if (p->drive_cap < ns) {
    if (p->d_drive) {
      HIPTRY(hipStreamSynchronize(st));
      if (p->hook.free)
        p->hook.free(p->hook.ctx, p->d_drive, (void*)p->home);
      else
        HIPTRY(hipFree(p->d_drive));
      p->d_drive = nullptr;
      p->drive_cap = 0;
    }
    if (dalloc(p, &p->d_drive, ns * sizeof(double)) != hipSuccess) {
      (void)hipGetLastError();
      return fail(SOP_ERR_NOMEM, "device allocation failed for the drive samples");
    }
    p->drive_cap = ns;
  }
  HIPTRY(hipMemcpyAsync(p->d_drive, drive, ns * sizeof(double), hipMemcpyHostToDevice, st));
  // one action at a time, each potential action with its own V = V0 + s D
  sop::DevView d = p->dv;
  d.graphs = nullptr;
  d.nact = 1;
  const size_t tab =
      (size_t)(p->S * (p->S + 1) / 2) * p->npts * p->csize * (p->dtype == SOP_C128 ? 1 : 2);
  // formation bytes per potential action: V0 and D read, the table written
  const double fbytes =
      (2.0 * (p->S * (p->S + 1) / 2) * sizeof(double) +
       (p->eig_form ? sop::eig_slots(p->S) * 16.0 : (double)tab / (double)p->npts)) *
      (double)p->npts;
  const int nact = (int)p->dv.hprog.size();
  const sop_status run = [&]() -> sop_status {
  for (int64_t n = 0; n < nsteps; ++n) {
    int v = 0;
    for (int a = 0; a < nact;) {
      const int code = p->dv.hprog[a];
      // a potential action runs together with the kinetic action after it
      // (on 3D grids inside that action's z-pass, as in a static step); a
      // potential action with no kinetic action after it in the step runs
      // alone
      int na = 1;
      if ((code >> 16) == sop::OP_V) {
        // V = V0 + s D formed inside the table kernel (no V table written)
        const double* s_dev = p->d_drive + (size_t)n * nv + v++;
        sop::TimedLaunch tl(d, sop::KIND_OTHER, fbytes);
        if (p->eig_form) {
          HIPTRY(sop::form_eigq(d, p->d_vbase, p->tile, p->d_vexp, p->d_dv, s_dev));
        } else {  // only the table this action reads
          const int idx = code & 0xffff;
          HIPTRY(sop::form_vexp(d, p->d_vbase, p->d_taus + idx, 1, p->tile,
                                (char*)p->d_vexp + (size_t)idx * tab, p->d_dv, s_dev));
        }
        if (a + 1 < nact && (p->dv.hprog[a + 1] >> 16) == sop::OP_T) na = 2;
      }
      d.prog = p->d_prog + a;
      d.nact = na;
      d.hprog.assign(p->dv.hprog.begin() + a, p->dv.hprog.begin() + a + na);
      if (p->ndim == 1)
        HIPTRY(sop::k1d_propagate(d, psi, 1, 0));
      else
        HIPTRY(sop::k3d_propagate(d, psi, 1, 0));
      a += na;
    }
  }
  return SOP_OK;
  }();
  // back to the tables of the plan's own V (its V-table was not touched), on
  // every exit path: a failed action must not leave the driven tables behind
  const hipError_t ef = form_tables(p);
  const hipError_t es = hipStreamSynchronize(st);
  if (run != SOP_OK) return run;  // the loop's failure text is kept
  HIPTRY(ef);
  HIPTRY(es);
  return SOP_OK;
}

sop_status sop_plan_update_v(sop_plan* p, const double* vtable) {
  if (!p || !vtable) return fail(SOP_ERR_INVALID, "NULL argument");
  const int NE = p->S * (p->S + 1) / 2;
  const size_t nv = (size_t)NE * p->npts;
  for (size_t i = 0; i < nv; ++i)
    if (!std::isfinite(vtable[i])) return fail(SOP_ERR_INVALID, "vtable must be finite");
  const double vb = p->eig_form ? gershgorin_bound(vtable, p->S, p->npts) : 0.0;
  if (p->eig_form && !phases_fit(p, param_bound(p, vb, p->theta.data())))
    return fail(SOP_ERR_UNSUPPORTED,
                "this V-table takes the phases tau*lambda beyond the eigen form's range");
  hipStream_t st = p->dv.stream;
  const size_t vbytes = nv * sizeof(double);
  if (p->nparams > 0) {
    HIPTRY(hipMemcpyAsync(p->d_vbase, vtable, vbytes, hipMemcpyHostToDevice, st));
    HIPTRY(sop::set_vparams(p->dv, p->d_vraw, p->d_vbase, p->d_dv, p->d_theta, p->nparams));
  } else {
    HIPTRY(hipMemcpyAsync(p->d_vraw, vtable, vbytes, hipMemcpyHostToDevice, st));
  }
  HIPTRY(form_tables(p));
  if (p->d_eig) HIPTRY(sop::form_eig(p->dv, p->d_vraw, p->tile, p->d_eig));
  HIPTRY(hipStreamSynchronize(st));
  if (p->eig_form) p->vbound = vb;
  return SOP_OK;
}

namespace {

struct AdjLayout {
  size_t psi = 0, qacc = 0, ckpt = 0, total = 0;
  int64_t ncp = 0;
};

sop_status adjoint_check(const sop_plan* p, int64_t nsteps, int K, AdjLayout* lay) {
  if (!p) return fail(SOP_ERR_INVALID, "plan is NULL");
  if (nsteps < 1 || K < 1) return fail(SOP_ERR_INVALID, "nsteps and K must be >= 1");
  if (p->nparams == 0) return fail(SOP_ERR_STATE, "plan has no parameters (nparams = 0)");
  if (!p->d_eig) return fail(SOP_ERR_UNSUPPORTED, "the adjoint needs an FP64 3D plan with n in {32, 64, 128, 256}");
  const size_t sb = (size_t)p->S * p->npts * sizeof(double) * 2;
  lay->ncp = (nsteps + K - 1) / K;
  lay->psi = 0;                                   // psi then lambda: 2 * sb
  lay->qacc = 2 * sb;                             // NE * npts doubles
  const size_t qb = (size_t)p->S * (p->S + 1) / 2 * p->npts * sizeof(double);
  lay->ckpt = lay->qacc + ((qb + 255) / 256) * 256;
  lay->total = lay->ckpt + (size_t)lay->ncp * sb;
  return SOP_OK;
}

}  // namespace

sop_status sop_adjoint_workspace_bytes(const sop_plan* p, int64_t nsteps, int K, size_t* bytes) {
  if (!bytes) return fail(SOP_ERR_INVALID, "bytes is NULL");
  AdjLayout lay;
  sop_status st = adjoint_check(p, nsteps, K, &lay);
  if (st != SOP_OK) return st;
  *bytes = lay.total;
  return SOP_OK;
}

sop_status sop_adjoint_forward(sop_plan* p, const void* psi0, int64_t nsteps, int K, void* ws,
                               double* pops_out) {
  AdjLayout lay;
  sop_status st = adjoint_check(p, nsteps, K, &lay);
  if (st != SOP_OK) return st;
  if (!psi0 || !ws || !pops_out) return fail(SOP_ERR_INVALID, "NULL argument");
  hipStream_t s = p->dv.stream;
  char* w = (char*)ws;
  const size_t sb = (size_t)p->S * p->npts * sizeof(double) * 2;
  HIPTRY(hipMemcpyAsync(w + lay.psi, psi0, sb, hipMemcpyDeviceToDevice, s));
  int64_t done = 0;
  for (int64_t c = 0; done < nsteps; ++c) {
    HIPTRY(hipMemcpyAsync(w + lay.ckpt + (size_t)c * sb, w + lay.psi, sb, hipMemcpyDeviceToDevice, s));
    const int64_t k = std::min<int64_t>(K, nsteps - done);
    HIPTRY(sop::k3d_propagate(p->dv, w + lay.psi, k, 0));
    done += k;
  }
  HIPTRY(sop::pops_reduce(p->dv, w + lay.psi, p->d_vraw, p->d_part, p->d_out));
  double raw[8];
  HIPTRY(hipMemcpyAsync(raw, p->d_out, (p->S + 1) * sizeof(double), hipMemcpyDeviceToHost, s));
  HIPTRY(hipStreamSynchronize(s));
  for (int q = 0; q < p->S; ++q) pops_out[q] = raw[q] * p->dV;
  return SOP_OK;
}

sop_status sop_adjoint_backward(sop_plan* p, int64_t nsteps, int K, const double* weights,
                                void* ws, double* grad_out) {
  AdjLayout lay;
  sop_status st = adjoint_check(p, nsteps, K, &lay);
  if (st != SOP_OK) return st;
  if (!weights || !ws || !grad_out) return fail(SOP_ERR_INVALID, "NULL argument");
  for (int q = 0; q < p->S; ++q)
    if (!std::isfinite(weights[q])) return fail(SOP_ERR_INVALID, "weights must be finite");
  hipStream_t s = p->dv.stream;
  char* w = (char*)ws;
  const size_t sb = (size_t)p->S * p->npts * sizeof(double) * 2;
  HIPTRY(hipMemcpyAsync(p->d_w, weights, p->S * sizeof(double), hipMemcpyHostToDevice, s));
  HIPTRY(sop::adjoint_seed(p->dv, w + lay.psi + sb, w + lay.psi, p->d_w, (double*)(w + lay.qacc)));
  sop::AdjointView a;
  a.stacked = w + lay.psi;
  a.eig = p->d_eig;
  a.qacc = (double*)(w + lay.qacc);
  a.taus = p->d_taus;
  a.checkpoints = w + lay.ckpt;
  HIPTRY(sop::k3d_adjoint_backward(p->dv, a, nsteps, K));
  HIPTRY(sop::grad_reduce(p->dv, a.qacc, sop::k3d_adjoint_cols(p->n[0]), p->d_dv, p->nparams,
                          p->d_part, p->d_out));
  double raw[sop::kMaxParams];
  HIPTRY(hipMemcpyAsync(raw, p->d_out, p->nparams * sizeof(double), hipMemcpyDeviceToHost, s));
  HIPTRY(hipStreamSynchronize(s));
  for (int k = 0; k < p->nparams; ++k) grad_out[k] = 2.0 * p->dV * raw[k];
  return SOP_OK;
}

sop_status sop_adjoint(sop_plan* p, const void* psi0, int64_t nsteps, int K,
                       const double* weights, void* ws, double* pops_out, double* grad_out) {
  if (!pops_out || !grad_out) return fail(SOP_ERR_INVALID, "NULL argument");
  std::vector<double> pops(p ? (size_t)p->S : 0), grad(p ? (size_t)p->nparams : 0);
  sop_status st = sop_adjoint_forward(p, psi0, nsteps, K, ws, pops.data());
  if (st != SOP_OK) return st;
  st = sop_adjoint_backward(p, nsteps, K, weights, ws, grad.data());
  if (st != SOP_OK) return st;
  std::copy(pops.begin(), pops.end(), pops_out);
  std::copy(grad.begin(), grad.end(), grad_out);
  return SOP_OK;
}

sop_status sop_plan_set_option(sop_plan* p, int option, int value) {
  if (!p) return fail(SOP_ERR_INVALID, "plan is NULL");
  switch (option) {
    case SOP_OPT_GRAPHS:
      p->use_graphs = value != 0;
      p->dv.graphs = (p->use_graphs && p->graphs) ? p->graphs : nullptr;
      return SOP_OK;
    case SOP_OPT_PLANE_PASS:
      if (p->graphs) {  // captured segments hold the old pass sequence
        HIPTRY(hipStreamSynchronize(p->dv.stream));
        p->graphs->clear();
      }
      p->dv.plane = value != 0;
      return SOP_OK;
    default:
      return fail(SOP_ERR_INVALID, "unknown option");
  }
}

sop_status sop_plan_set_timing(sop_plan* p, int enable) {
  if (!p) return fail(SOP_ERR_INVALID, "plan is NULL");
  if (enable) {
    if (!p->timer) {
      p->timer = new (std::nothrow) sop::Timer();
      if (!p->timer) return fail(SOP_ERR_NOMEM, "host allocation failed");
    }
    p->dv.timer = p->timer;
  } else {
    p->dv.timer = nullptr;
  }
  return SOP_OK;
}

sop_status sop_timing_read(sop_plan* p, double* ms, int64_t* counts, double* bytes) {
  if (!p || !ms || !counts || !bytes) return fail(SOP_ERR_INVALID, "NULL argument");
  for (int k = 0; k < SOP_KIND_COUNT; ++k) {
    ms[k] = 0;
    counts[k] = 0;
    bytes[k] = 0;
  }
  if (!p->timer) return SOP_OK;
  HIPTRY(hipStreamSynchronize(p->dv.stream));
  for (const auto& r : p->timer->recs) {
    float t = 0;
    HIPTRY(hipEventElapsedTime(&t, r.a, r.b));
    ms[r.kind] += t;
    counts[r.kind] += 1;
    bytes[r.kind] += r.bytes;
  }
  p->timer->recs.clear();
  p->timer->used = 0;
  return SOP_OK;
}

}  // extern "C"
