// soref.cpp -- plain FP64 CPU oracle for the composed split-operator propagator.
//
// TEST INFRASTRUCTURE ONLY.  Nothing in the product path links, loads or calls
// this file; only the tests, the smoke check and the CPU-baseline leg of the
// benchmark do.  It shares no source with the HIP library: its composition
// recursion, pruning, dedupe, FFT, Jacobi eigensolver, exponentials and
// observables are written here from the paper, for readability over speed.
//
// Paper: Roulet, Choi, Vanicek, "Efficient geometric integrators for
// nonadiabatic quantum dynamics. II. The diabatic representation"
// (arXiv:1903.04946).  Citations name the section / equation label / table.
//
// Conventions (readings of points the paper leaves open are listed in the
// design notes of the repository):
//   * state psi: complex128, layout [S][n_0]...[n_{D-1}], last axis fastest;
//   * grid: periodic, x_j = lo + j*dx, dx = (hi-lo)/n (right endpoint excluded);
//   * momentum p_k = hbar * 2*pi*k'/(n*dx), k' = k for k < n/2 else k - n;
//   * forward FFT exp(-2 pi i jk/n) unnormalised, inverse exp(+2 pi i jk/n)/n;
//   * V-table: real symmetric S x S matrix per point, packed upper triangle
//     (V00, V01, .., V0,S-1, V11, ..), array [S(S+1)/2][npts];
//   * kinetic energy T(p) = sum_d p_d^2 / (2 m_d)  (Eq. diab_mol_ham).
//
// OpenMP (when enabled at build time) only spreads independent pencils and
// grid points over threads; every number is the same for any thread count.

#include <algorithm>
#include <chrono>
#include <cmath>
#include <complex>
#include <cstdint>
#include <cstring>
#include <map>
#include <mutex>
#include <vector>
#ifdef _OPENMP
#include <omp.h>
#endif

typedef std::complex<double> cd;
typedef long double ld;

static const ld PI_L = 3.141592653589793238462643383279502884197L;

extern "C" {

// Problem description shared with the ctypes wrapper (oracle/oracle.py).
struct orc_problem {
  int ndim;
  int n[3];
  double lo[3];
  double hi[3];
  int nsurf;
  double inv_mass[3];
  double hbar;
  const double* vtable;  // [S(S+1)/2][npts], packed upper triangle
};

}  // extern "C"

// ---------------------------------------------------------------------------
// Composition coefficients (Sec. "Symmetric composition schemes"; the
// fourth-order instances are Eqs. triple_jump_fourth_order_so and
// suzukis_fractals_fourth_order_so; recursion per Sec. "Compositions of
// split-operator algorithms": "both composition procedures can be applied
// recursively").
//
// Raising the order p -> p+2: the triple jump uses the symmetric outer
// coefficients (c, 1-2c, c) with c = 1/(2 - 2^{1/(p+1)}); Suzuki's fractal
// uses (c, c, 1-4c, c, c) with c = 1/(4 - 4^{1/(p+1)}).  U_{p+2}(dt) =
// U_p(g_M dt) ... U_p(g_1 dt): each outer stage scales the whole inner
// sequence, so the flattened list is outer-major.
// ---------------------------------------------------------------------------
enum { ORC_STRANG = 0, ORC_TRIPLE_JUMP = 1, ORC_SUZUKI = 2 };
enum { ORC_VTV = 0, ORC_TVT = 1, ORC_VT = 2, ORC_TV = 3 };

static bool gammas_ld(int scheme, int order, std::vector<ld>& g) {
  g.assign(1, 1.0L);
  if (order < 2 || (order % 2) != 0) return false;
  if (scheme == ORC_STRANG) return order == 2;
  if (scheme != ORC_TRIPLE_JUMP && scheme != ORC_SUZUKI) return false;
  for (int p = 2; p < order; p += 2) {
    std::vector<ld> outer;
    if (scheme == ORC_TRIPLE_JUMP) {
      ld c = 1.0L / (2.0L - powl(2.0L, 1.0L / (ld)(p + 1)));
      outer = {c, 1.0L - 2.0L * c, c};
    } else {
      ld c = 1.0L / (4.0L - powl(4.0L, 1.0L / (ld)(p + 1)));
      outer = {c, c, 1.0L - 4.0L * c, c, c};
    }
    std::vector<ld> next;
    for (ld o : outer)
      for (ld x : g) next.push_back(o * x);
    g.swap(next);
  }
  return true;
}

// Splitting sequence U = B(b_N)A(a_N) ... B(b_1)A(a_1), A(a_1) applied first
// (Sec. "Compositions of split-operator algorithms").  Each Strang stage with
// composition coefficient g contributes a = (g/2, g/2), b = (g, 0)
// (Eq. second_order_so scaled by g).  First-order splittings have a = b = (1).
// Pruning (Eq. merging_splitting_coeff_b_zero) removes each interior b_j = 0
// by merging a_j and a_{j+1}; the trailing b_N = 0 is the identity and is kept
// only as a zero entry.  The merged sums are formed in long double and rounded
// once.
static bool splitting_ld(int split, int scheme, int order, bool pruned,
                         std::vector<ld>& a, std::vector<ld>& b) {
  a.clear();
  b.clear();
  if (split == ORC_VT || split == ORC_TV) {
    if (order != 1) return false;
    a.push_back(1.0L);
    b.push_back(1.0L);
    return true;
  }
  if (split != ORC_VTV && split != ORC_TVT) return false;
  std::vector<ld> g;
  if (!gammas_ld(scheme, order, g)) return false;
  // unpruned sequence
  std::vector<ld> ua, ub;
  for (ld x : g) {
    ua.push_back(x / 2);
    ua.push_back(x / 2);
    ub.push_back(x);
    ub.push_back(0.0L);
  }
  if (!pruned) {
    a = ua;
    b = ub;
    return true;
  }
  // Apply the merge rule for every zero b_j with j != N, left to right.
  a = ua;
  b = ub;
  size_t j = 0;
  while (j + 1 < b.size()) {
    if (b[j] == 0.0L) {
      a[j] = a[j] + a[j + 1];
      a.erase(a.begin() + (long)j + 1);
      b.erase(b.begin() + (long)j);
    } else {
      ++j;
    }
  }
  return true;
}

// Unique coefficients and index arrays (Sec. "Pruning splitting coefficients",
// Eq. range_index_unq): a value joins an existing unique entry when the two
// agree to 1e-13 relative; the first occurrence is canonical.  Indices here
// are 0-based.  The oracle searches the whole sequence (the symmetric
// half-search of the paper is an optimisation it does not need).
static void dedupe(const std::vector<double>& v, std::vector<double>& unq,
                   std::vector<int>& idx) {
  unq.clear();
  idx.clear();
  for (double x : v) {
    int found = -1;
    for (size_t u = 0; u < unq.size(); ++u) {
      double scale = std::max(std::fabs(x), std::fabs(unq[u]));
      if (std::fabs(x - unq[u]) <= 1e-13 * scale) {
        found = (int)u;
        break;
      }
    }
    if (found < 0) {
      unq.push_back(x);
      found = (int)unq.size() - 1;
    }
    idx.push_back(found);
  }
}

// ---------------------------------------------------------------------------
// Discrete Fourier transform (Sec. "Dynamic Fourier method").
// Power-of-two lengths: iterative radix-2 Cooley-Tukey with bit reversal,
// twiddles exp(-2 pi i k/n) each evaluated in long double (no recurrence).
// Other lengths: the plain O(n^2) sum with long-double twiddles.
// ---------------------------------------------------------------------------
static std::mutex g_tw_mutex;
static std::map<int, std::vector<cd>> g_tw;  // n -> exp(-2 pi i k/n), k < n

static const std::vector<cd>& twiddles(int n) {
  std::lock_guard<std::mutex> lk(g_tw_mutex);
  auto it = g_tw.find(n);
  if (it != g_tw.end()) return it->second;
  std::vector<cd> w(n);
  for (int k = 0; k < n; ++k) {
    ld ang = -2.0L * PI_L * (ld)k / (ld)n;
    w[k] = cd((double)cosl(ang), (double)sinl(ang));
  }
  return g_tw.emplace(n, std::move(w)).first->second;
}

static bool is_pow2(int n) { return n > 0 && (n & (n - 1)) == 0; }

// In-place transform of a contiguous buffer of length n.
static void fft_buffer(cd* a, int n, bool inverse, const std::vector<cd>& w) {
  if (is_pow2(n)) {
    // bit-reversal permutation
    for (int i = 1, j = 0; i < n; ++i) {
      int bit = n >> 1;
      for (; j & bit; bit >>= 1) j ^= bit;
      j ^= bit;
      if (i < j) std::swap(a[i], a[j]);
    }
    for (int len = 2; len <= n; len <<= 1) {
      int half = len / 2, step = n / len;
      for (int i = 0; i < n; i += len) {
        for (int k = 0; k < half; ++k) {
          cd tw = w[k * step];
          if (inverse) tw = std::conj(tw);
          cd u = a[i + k];
          cd v = a[i + k + half] * tw;
          a[i + k] = u + v;
          a[i + k + half] = u - v;
        }
      }
    }
  } else {
    std::vector<cd> out(n);
    for (int k = 0; k < n; ++k) {
      cd s(0.0, 0.0);
      for (int j = 0; j < n; ++j) {
        cd tw = w[(int)(((int64_t)j * k) % n)];
        if (inverse) tw = std::conj(tw);
        s += a[j] * tw;
      }
      out[k] = s;
    }
    std::copy(out.begin(), out.end(), a);
  }
  if (inverse) {
    double s = 1.0 / (double)n;
    for (int i = 0; i < n; ++i) a[i] *= s;
  }
}

struct Grid {
  int ndim = 1;
  int n[3] = {1, 1, 1};
  double dx[3] = {1, 1, 1};
  int64_t npts = 1;
  double dV = 1;
  int S = 1;
  double inv_mass[3] = {1, 1, 1};
  double hbar = 1;
  int64_t stride[3] = {1, 1, 1};  // element stride of each axis
};

static bool make_grid(const orc_problem* p, Grid& g) {
  if (!p || p->ndim < 1 || p->ndim > 3 || p->nsurf < 1 || p->nsurf > 8) return false;
  if (!(p->hbar > 0)) return false;
  g.ndim = p->ndim;
  g.S = p->nsurf;
  g.hbar = p->hbar;
  g.npts = 1;
  g.dV = 1;
  for (int d = 0; d < 3; ++d) {
    g.n[d] = 1;
    g.dx[d] = 1;
    g.inv_mass[d] = 0;
  }
  for (int d = 0; d < p->ndim; ++d) {
    if (p->n[d] < 1) return false;
    if (!(p->hi[d] > p->lo[d])) return false;
    g.n[d] = p->n[d];
    g.dx[d] = (p->hi[d] - p->lo[d]) / (double)p->n[d];
    g.inv_mass[d] = p->inv_mass[d];
    g.npts *= p->n[d];
    g.dV *= g.dx[d];
  }
  int64_t s = 1;
  for (int d = p->ndim - 1; d >= 0; --d) {
    g.stride[d] = s;
    s *= g.n[d];
  }
  return true;
}

// Forward (inverse=false) or inverse transform of every surface along every
// axis of a state [S][npts].
static void fft_state(const Grid& g, cd* psi, bool inverse) {
  for (int d = 0; d < g.ndim; ++d) {
    const int n = g.n[d];
    if (n == 1) continue;
    const std::vector<cd>& w = twiddles(n);
    const int64_t st = g.stride[d];
    const int64_t npencil = g.npts / n;
    const int64_t total = npencil * g.S;
#pragma omp parallel
    {
      std::vector<cd> buf(n);
#pragma omp for schedule(static)
      for (int64_t q = 0; q < total; ++q) {
        int64_t s = q / npencil, r = q % npencil;
        // r enumerates the pencil: split into (outer, inner) around axis d
        int64_t inner = r % st, outer = r / st;
        cd* base = psi + s * g.npts + outer * st * n + inner;
        for (int j = 0; j < n; ++j) buf[j] = base[(int64_t)j * st];
        fft_buffer(buf.data(), n, inverse, w);
        for (int j = 0; j < n; ++j) base[(int64_t)j * st] = buf[j];
      }
    }
  }
}

// Momentum of index k on an axis with n points and spacing dx.
static double momentum(const Grid& g, int d, int k) {
  int n = g.n[d];
  int kk = (k < n / 2) ? k : k - n;
  return g.hbar * 2.0 * (double)PI_L * (double)kk / ((double)n * g.dx[d]);
}

// T(p) at the flat momentum index (Eq. diab_mol_ham: p^T m^{-1} p / 2).
static double kinetic_energy_at(const Grid& g, int64_t flat) {
  double t = 0;
  for (int d = 0; d < g.ndim; ++d) {
    int k = (int)((flat / g.stride[d]) % g.n[d]);
    double p = momentum(g, d, k);
    t += 0.5 * g.inv_mass[d] * p * p;
  }
  return t;
}

// ---------------------------------------------------------------------------
// Cyclic Jacobi eigensolver for a real symmetric n x n matrix (Sec.
// "Molecular Hamiltonian in the diabatic basis": the potential exponential is
// obtained from the diagonalised matrix; for 2 x 2 one rotation is exact).
// A is row-major and destroyed; on return A's diagonal holds the eigenvalues
// and R's columns are the eigenvectors (V = R diag(lam) R^T).
// A rotation annihilates a_pq; an element negligible next to both diagonal
// entries is set to zero.  Sweeps repeat until every off-diagonal is zero.
// ---------------------------------------------------------------------------
static void jacobi_eigen(int n, std::vector<double>& A, std::vector<double>& R,
                         std::vector<double>& lam) {
  R.assign((size_t)n * n, 0.0);
  for (int i = 0; i < n; ++i) R[(size_t)i * n + i] = 1.0;
  auto a = [&](int i, int j) -> double& { return A[(size_t)i * n + j]; };
  for (int sweep = 0; sweep < 100; ++sweep) {
    bool any = false;
    for (int p = 0; p < n - 1; ++p) {
      for (int q = p + 1; q < n; ++q) {
        double apq = a(p, q);
        if (apq == 0.0) continue;
        double app = a(p, p), aqq = a(q, q);
        if (std::fabs(app) + 100.0 * std::fabs(apq) == std::fabs(app) &&
            std::fabs(aqq) + 100.0 * std::fabs(apq) == std::fabs(aqq) && sweep > 2) {
          a(p, q) = 0.0;
          a(q, p) = 0.0;
          continue;
        }
        any = true;
        double theta = (aqq - app) / (2.0 * apq);
        double t;
        if (std::fabs(theta) > 1e150) {
          t = 0.5 / theta;
        } else {
          t = 1.0 / (std::fabs(theta) + std::sqrt(theta * theta + 1.0));
          if (theta < 0) t = -t;
        }
        double c = 1.0 / std::sqrt(t * t + 1.0);
        double s = t * c;
        for (int r = 0; r < n; ++r) {
          if (r == p || r == q) continue;
          double arp = a(r, p), arq = a(r, q);
          double nrp = c * arp - s * arq;
          double nrq = s * arp + c * arq;
          a(r, p) = nrp;
          a(p, r) = nrp;
          a(r, q) = nrq;
          a(q, r) = nrq;
        }
        a(p, p) = app - t * apq;
        a(q, q) = aqq + t * apq;
        a(p, q) = 0.0;
        a(q, p) = 0.0;
        for (int r = 0; r < n; ++r) {
          double vrp = R[(size_t)r * n + p], vrq = R[(size_t)r * n + q];
          R[(size_t)r * n + p] = c * vrp - s * vrq;
          R[(size_t)r * n + q] = s * vrp + c * vrq;
        }
      }
    }
    if (!any) break;
  }
  lam.resize(n);
  for (int i = 0; i < n; ++i) lam[i] = a(i, i);
}

static int packed_index(int S, int i, int j) {
  if (i > j) std::swap(i, j);
  // rows 0..i-1 hold S, S-1, ..., S-i+1 entries
  return i * S - (i * (i - 1)) / 2 + (j - i);
}

// Per-point eigen-decomposition of V(x), cached for the propagation.
struct PotentialEigen {
  int S = 0;
  int64_t npts = 0;
  std::vector<double> R;    // [npts][S][S] (columns eigenvectors)
  std::vector<double> lam;  // [npts][S]
};

static void potential_eigen(const Grid& g, const double* vtable, PotentialEigen& pe) {
  const int S = g.S;
  pe.S = S;
  pe.npts = g.npts;
  pe.R.assign((size_t)g.npts * S * S, 0.0);
  pe.lam.assign((size_t)g.npts * S, 0.0);
#pragma omp parallel
  {
    std::vector<double> A((size_t)S * S), R, lam;
#pragma omp for schedule(static)
    for (int64_t x = 0; x < g.npts; ++x) {
      for (int i = 0; i < S; ++i)
        for (int j = 0; j < S; ++j)
          A[(size_t)i * S + j] = vtable[(int64_t)packed_index(S, i, j) * g.npts + x];
      jacobi_eigen(S, A, R, lam);
      std::copy(R.begin(), R.end(), pe.R.begin() + (size_t)x * S * S);
      std::copy(lam.begin(), lam.end(), pe.lam.begin() + (size_t)x * S);
    }
  }
}

// U = R diag(exp(-i lam tau / hbar)) R^T at one point, written to U[S][S].
static void point_exponential(int S, const double* R, const double* lam, double tau,
                              double hbar, cd* U) {
  cd e[8];
  for (int l = 0; l < S; ++l) {
    double ph = -lam[l] * tau / hbar;
    e[l] = cd(std::cos(ph), std::sin(ph));
  }
  for (int i = 0; i < S; ++i)
    for (int j = 0; j < S; ++j) {
      cd s(0, 0);
      for (int l = 0; l < S; ++l) s += R[i * S + l] * e[l] * R[j * S + l];
      U[i * S + j] = s;
    }
}

// Action of the potential evolution operator exp(-i tau V(q)/hbar): the
// S x S unitary applied to the surface vector at every grid point
// (Sec. "Dynamic Fourier method", Sec. "Molecular Hamiltonian...").
static void potential_action(const Grid& g, const PotentialEigen& pe, double tau, cd* psi) {
  const int S = g.S;
#pragma omp parallel
  {
    std::vector<cd> U((size_t)S * S), v(S), w(S);
#pragma omp for schedule(static)
    for (int64_t x = 0; x < g.npts; ++x) {
      point_exponential(S, &pe.R[(size_t)x * S * S], &pe.lam[(size_t)x * S], tau, g.hbar,
                        U.data());
      for (int s = 0; s < S; ++s) v[s] = psi[s * g.npts + x];
      for (int i = 0; i < S; ++i) {
        cd acc(0, 0);
        for (int j = 0; j < S; ++j) acc += U[i * S + j] * v[j];
        w[i] = acc;
      }
      for (int s = 0; s < S; ++s) psi[s * g.npts + x] = w[s];
    }
  }
}

// Action of the kinetic evolution operator exp(-i tau T(p)/hbar): forward
// FFT, multiply in the momentum representation, inverse FFT.
static void kinetic_action(const Grid& g, double tau, cd* psi) {
  fft_state(g, psi, false);
#pragma omp parallel for schedule(static)
  for (int64_t k = 0; k < g.npts; ++k) {
    double ph = -tau * kinetic_energy_at(g, k) / g.hbar;
    cd f(std::cos(ph), std::sin(ph));
    for (int s = 0; s < g.S; ++s) psi[s * g.npts + k] *= f;
  }
  fft_state(g, psi, true);
}

// One operator action: which physical operator plays A and B depends on the
// splitting (VTV and TV apply V first, i.e. A = V; TVT and VT apply T first).
static bool a_is_potential(int split) { return split == ORC_VTV || split == ORC_TV; }

extern "C" {

// ---------------------------------------------------------------- coefficients
// Composition coefficients gamma_1..gamma_M rounded to double.  Returns M,
// or -1 on invalid input / insufficient capacity.
int orc_gammas(int scheme, int order, double* out, int cap) {
  std::vector<ld> g;
  if (!gammas_ld(scheme, order, g)) return -1;
  if ((int)g.size() > cap) return -1;
  for (size_t i = 0; i < g.size(); ++i) out[i] = (double)g[i];
  return (int)g.size();
}

// Splitting coefficients a_j, b_j (j = 1..N) of the unpruned (pruned = 0) or
// pruned (pruned = 1) sequence.  Returns N or -1.
int orc_splitting(int split, int scheme, int order, int pruned, double* a, double* b,
                  int cap) {
  std::vector<ld> la, lb;
  if (!splitting_ld(split, scheme, order, pruned != 0, la, lb)) return -1;
  if ((int)la.size() > cap) return -1;
  for (size_t i = 0; i < la.size(); ++i) {
    a[i] = (double)la[i];
    b[i] = (double)lb[i];
  }
  return (int)la.size();
}

// Unique coefficients of the pruned sequence.  a_unq/b_unq receive the
// unique values, ia/ib (length N) the 0-based indices; counts[0..3] =
// (N, N_A, N_B, ...) -> counts = {N, n_a_unq, n_b_unq, n_b_nonzero}.
// Zero b entries (the trailing identity) are not entered in b_unq; their
// index is -1.  Returns 0 or -1.
int orc_unique(int split, int scheme, int order, double* a_unq, double* b_unq, int* ia,
               int* ib, int cap, int* counts) {
  std::vector<ld> la, lb;
  if (!splitting_ld(split, scheme, order, true, la, lb)) return -1;
  if ((int)la.size() > cap) return -1;
  std::vector<double> a(la.begin(), la.end()), bnz;
  std::vector<int> bpos;
  for (size_t j = 0; j < lb.size(); ++j)
    if (lb[j] != 0.0L) {
      bnz.push_back((double)lb[j]);
      bpos.push_back((int)j);
    }
  std::vector<double> ua, ub;
  std::vector<int> xa, xb;
  dedupe(a, ua, xa);
  dedupe(bnz, ub, xb);
  for (size_t i = 0; i < ua.size(); ++i) a_unq[i] = ua[i];
  for (size_t i = 0; i < ub.size(); ++i) b_unq[i] = ub[i];
  for (size_t j = 0; j < la.size(); ++j) {
    ia[j] = xa[j];
    ib[j] = -1;
  }
  for (size_t q = 0; q < bpos.size(); ++q) ib[bpos[q]] = xb[q];
  counts[0] = (int)la.size();
  counts[1] = (int)ua.size();
  counts[2] = (int)ub.size();
  counts[3] = (int)bnz.size();
  return 0;
}

// ---------------------------------------------------------------- FFT
// In-place 1D transform of n complex values (interleaved re, im).
int orc_fft(int n, int inverse, double* data) {
  if (n < 1) return -1;
  fft_buffer(reinterpret_cast<cd*>(data), n, inverse != 0, twiddles(n));
  return 0;
}

// ---------------------------------------------------------------- exponential
// U = exp(-i tau V / hbar) for one real symmetric S x S matrix V (row-major),
// written as S x S complex (interleaved).  Uses the Jacobi decomposition.
int orc_expm_potential(int S, const double* V, double tau, double hbar, double* U) {
  if (S < 1 || S > 64) return -1;
  std::vector<double> A(V, V + (size_t)S * S), R, lam;
  jacobi_eigen(S, A, R, lam);
  point_exponential(S, R.data(), lam.data(), tau, hbar, reinterpret_cast<cd*>(U));
  return 0;
}

// Eigen-decomposition of a real symmetric matrix (for pins of the solver).
int orc_eigh(int n, const double* A_in, double* lam_out, double* R_out) {
  if (n < 1) return -1;
  std::vector<double> A(A_in, A_in + (size_t)n * n), R, lam;
  jacobi_eigen(n, A, R, lam);
  std::copy(lam.begin(), lam.end(), lam_out);
  std::copy(R.begin(), R.end(), R_out);
  return 0;
}

// ---------------------------------------------------------------- propagation
// The step loop shared by orc_propagate and orc_propagate_timed: nsteps time
// steps of the sequence (a, b) with the actions run A(a_1), B(b_1), A(a_2),
// ... left to right in time (Sec. "Compositions of split-operator
// algorithms"); a zero b is skipped.  No merging across steps.
static void step_loop(const Grid& g, const PotentialEigen& pe, bool aV, const std::vector<double>& a,
                      const std::vector<double>& b, double dt, int64_t nsteps, cd* psi) {
  for (int64_t step = 0; step < nsteps; ++step) {
    for (size_t j = 0; j < a.size(); ++j) {
      if (aV)
        potential_action(g, pe, a[j] * dt, psi);
      else
        kinetic_action(g, a[j] * dt, psi);
      if (b[j] != 0.0) {
        if (aV)
          kinetic_action(g, b[j] * dt, psi);
        else
          potential_action(g, pe, b[j] * dt, psi);
      }
    }
  }
}

// Propagates psi in place by nsteps time steps of size dt (negative dt runs
// backwards in time).  pruned = 0 applies every Strang stage separately
// (A(g/2) B(g) A(g/2)); pruned = 1 applies the merged sequence.  Returns 0 or
// -1.  When seconds is not null it receives the wall time of the step loop
// alone (std::chrono::steady_clock; the per-point eigen-decomposition done
// before the loop is excluded), for timing the oracle as a CPU baseline.
static int propagate_impl(const orc_problem* prob, int split, int scheme, int order, double dt,
                          int64_t nsteps, int pruned, double* psi_io, double* seconds) {
  Grid g;
  if (!make_grid(prob, g) || !prob->vtable || nsteps < 0) return -1;
  std::vector<ld> la, lb;
  if (!splitting_ld(split, scheme, order, pruned != 0, la, lb)) return -1;
  std::vector<double> a(la.begin(), la.end()), b(lb.begin(), lb.end());
  PotentialEigen pe;
  potential_eigen(g, prob->vtable, pe);
  cd* psi = reinterpret_cast<cd*>(psi_io);
  const auto t0 = std::chrono::steady_clock::now();
  step_loop(g, pe, a_is_potential(split), a, b, dt, nsteps, psi);
  if (seconds)
    *seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  return 0;
}

int orc_propagate(const orc_problem* prob, int split, int scheme, int order, double dt,
                  int64_t nsteps, int pruned, double* psi_io) {
  return propagate_impl(prob, split, scheme, order, dt, nsteps, pruned, psi_io, nullptr);
}

// Propagation by a composition with given coefficients gamma_1..gamma_M
// (Sec. "Symmetric composition schemes"): every time step applies the Strang
// stages S(gamma_1 dt), ..., S(gamma_M dt) in turn, each one as A(gamma/2)
// B(gamma) A(gamma/2) with nothing merged (Eq. second_order_so scaled by
// gamma).  split is VTV or TVT.  The coefficients are taken as given: no
// symmetry or sum is required here.  Returns 0 or -1.
int orc_propagate_gamma(const orc_problem* prob, int split, int M, const double* gamma,
                        double dt, int64_t nsteps, double* psi_io) {
  Grid g;
  if (!make_grid(prob, g) || !prob->vtable || nsteps < 0 || M < 1 || !gamma) return -1;
  if (split != ORC_VTV && split != ORC_TVT) return -1;
  PotentialEigen pe;
  potential_eigen(g, prob->vtable, pe);
  cd* psi = reinterpret_cast<cd*>(psi_io);
  const bool aV = a_is_potential(split);
  auto A = [&](double tau) {
    if (aV)
      potential_action(g, pe, tau, psi);
    else
      kinetic_action(g, tau, psi);
  };
  auto B = [&](double tau) {
    if (aV)
      kinetic_action(g, tau, psi);
    else
      potential_action(g, pe, tau, psi);
  };
  for (int64_t step = 0; step < nsteps; ++step)
    for (int k = 0; k < M; ++k) {
      A(0.5 * gamma[k] * dt);
      B(gamma[k] * dt);
      A(0.5 * gamma[k] * dt);
    }
  return 0;
}

// Driven potential V(x, t) = V0(x) + s(t) D(x) (Sec. "Pruning splitting
// coefficients": a time-dependent operator is formed on the fly, at every
// action).  The v-th potential action of step n uses the drive value
// drive[n * nv + v] (nv potential actions per step); its exp(-i tau V/hbar)
// comes from a per-point eigen-decomposition of V0 + s D made for that
// action.  The caller chooses the times at which s is sampled.
int orc_propagate_driven(const orc_problem* prob, const double* dtable, int split, int scheme,
                         int order, double dt, int64_t nsteps, const double* drive,
                         double* psi_io) {
  Grid g;
  if (!make_grid(prob, g) || !prob->vtable || !dtable || nsteps < 0) return -1;
  std::vector<ld> la, lb;
  if (!splitting_ld(split, scheme, order, true, la, lb)) return -1;
  std::vector<double> a(la.begin(), la.end()), b(lb.begin(), lb.end());
  const bool aV = a_is_potential(split);
  int64_t nv = 0;  // potential actions per step
  for (size_t j = 0; j < a.size(); ++j) nv += aV ? 1 : (b[j] != 0.0 ? 1 : 0);
  const int NE = g.S * (g.S + 1) / 2;
  const size_t ntab = (size_t)NE * g.npts;
  std::vector<double> vt(ntab);
  PotentialEigen pe;
  cd* psi = reinterpret_cast<cd*>(psi_io);
  auto potential = [&](double tau, double s) {
    for (size_t i = 0; i < ntab; ++i) vt[i] = prob->vtable[i] + s * dtable[i];
    potential_eigen(g, vt.data(), pe);
    potential_action(g, pe, tau, psi);
  };
  for (int64_t step = 0; step < nsteps; ++step) {
    int64_t v = 0;
    for (size_t j = 0; j < a.size(); ++j) {
      if (aV)
        potential(a[j] * dt, drive[step * nv + v++]);
      else
        kinetic_action(g, a[j] * dt, psi);
      if (b[j] != 0.0) {
        if (aV)
          kinetic_action(g, b[j] * dt, psi);
        else
          potential(b[j] * dt, drive[step * nv + v++]);
      }
    }
  }
  return 0;
}

// Trigonometric interpolation (Appendix B: a state on one grid is compared
// with a state on a grid of other range and density through the
// trigonometric interpolant of the one on the sparser grid).  Along one axis,
// the samples u_m at x_m = lo + m dx (n points, L = hi - lo) define
// c_k = (1/n) sum_m u_m exp(-2 pi i k m/n), and the interpolant at x is
// sum_{|k| < n/2} c_k exp(2 pi i k xi) + [n even] c_{n/2} cos(pi n xi),
// xi = (x - lo)/L; it is taken as zero where xi is outside [0, 1).  The 3D
// interpolant is this applied along every axis (the axes separate).  The
// destination points are x = lo_d + j (hi_d - lo_d)/n_d.  Sums and phases in
// long double.  psi arrays are [S][grid] complex (interleaved).  Returns 0 or -1.
static void interp_line(int n, double lo, double hi, const cd* u, int64_t su, int nd,
                        double lod, double hid, cd* out, int64_t so) {
  std::vector<std::complex<ld>> c(n);
  for (int k = 0; k < n; ++k) {
    std::complex<ld> acc = 0;
    for (int m = 0; m < n; ++m) {
      const ld ph = -2 * PI_L * (ld)(((int64_t)k * m) % n) / n;
      acc += std::complex<ld>(u[m * su].real(), u[m * su].imag()) *
             std::complex<ld>(cosl(ph), sinl(ph));
    }
    c[k] = acc / (ld)n;
  }
  const double dxd = (hid - lod) / nd;
  for (int j = 0; j < nd; ++j) {
    const double x = lod + j * dxd;
    const double xi = (x - lo) / (hi - lo);
    std::complex<ld> v = 0;
    if (xi >= 0.0 && xi < 1.0) {
      for (int k = -((n - 1) / 2); k <= (n - 1) / 2; ++k) {
        const ld ph = 2 * PI_L * (ld)k * (ld)xi;
        v += c[(k + n) % n] * std::complex<ld>(cosl(ph), sinl(ph));
      }
      if (n % 2 == 0) v += c[n / 2] * cosl(PI_L * (ld)n * (ld)xi);
    }
    out[j * so] = cd((double)v.real(), (double)v.imag());
  }
}

int orc_interpolate(int ndim, int S, const int* n_src, const double* lo_src, const double* hi_src,
                    const double* psi_src, const int* n_dst, const double* lo_dst,
                    const double* hi_dst, double* psi_dst) {
  if ((ndim != 1 && ndim != 3) || S < 1 || !psi_src || !psi_dst) return -1;
  int64_t cur[3] = {1, 1, 1};
  for (int a = 0; a < ndim; ++a) {
    if (n_src[a] < 1 || n_dst[a] < 1 || !(hi_src[a] > lo_src[a]) || !(hi_dst[a] > lo_dst[a]))
      return -1;
    cur[a] = n_src[a];
  }
  std::vector<cd> buf(reinterpret_cast<const cd*>(psi_src),
                      reinterpret_cast<const cd*>(psi_src) + S * cur[0] * cur[1] * cur[2]);
  // interpolate axis by axis, last (contiguous) axis first
  for (int a = ndim - 1; a >= 0; --a) {
    int64_t shape[3] = {cur[0], cur[1], cur[2]};
    int64_t nshape[3] = {cur[0], cur[1], cur[2]};
    nshape[a] = n_dst[a];
    int64_t stride[3] = {shape[1] * shape[2], shape[2], 1};
    int64_t nstride[3] = {nshape[1] * nshape[2], nshape[2], 1};
    const int64_t nblock = S * shape[0] * shape[1] * shape[2];
    std::vector<cd> next((size_t)S * nshape[0] * nshape[1] * nshape[2]);
    const int64_t per_s = shape[0] * shape[1] * shape[2];
    const int64_t nper_s = nshape[0] * nshape[1] * nshape[2];
    (void)nblock;
#pragma omp parallel for collapse(3) schedule(static)
    for (int s = 0; s < S; ++s)
      for (int64_t i0 = 0; i0 < (a == 0 ? 1 : shape[0]); ++i0)
        for (int64_t i1 = 0; i1 < (a == 1 || ndim == 1 ? 1 : shape[1]); ++i1)
          for (int64_t i2 = 0; i2 < (a == 2 || ndim == 1 ? 1 : shape[2]); ++i2) {
            const int64_t src_off = s * per_s + i0 * stride[0] + i1 * stride[1] + i2 * stride[2];
            const int64_t dst_off =
                s * nper_s + i0 * nstride[0] + i1 * nstride[1] + i2 * nstride[2];
            interp_line((int)shape[a], lo_src[a], hi_src[a], buf.data() + src_off, stride[a],
                        n_dst[a], lo_dst[a], hi_dst[a], next.data() + dst_off, nstride[a]);
          }
    buf.swap(next);
    cur[a] = n_dst[a];
  }
  std::copy(buf.begin(), buf.end(), reinterpret_cast<cd*>(psi_dst));
  return 0;
}

// orc_propagate with pruned = 1, and writes to *seconds the wall time of the
// step loop alone (the same loop, see propagate_impl).  Used to time the
// oracle as a CPU baseline.
int orc_propagate_timed(const orc_problem* prob, int split, int scheme, int order, double dt,
                        int64_t nsteps, double* psi_io, double* seconds) {
  if (!seconds) return -1;
  return propagate_impl(prob, split, scheme, order, dt, nsteps, 1, psi_io, seconds);
}

// Sets the number of threads of the OpenMP loops (n >= 1; no effect without
// OpenMP).  For timing the oracle single-threaded and on all cores.
int orc_set_threads(int n) {
  if (n < 1) return -1;
#ifdef _OPENMP
  omp_set_num_threads(n);
#endif
  return 0;
}

// Number of threads the OpenMP loops use (1 without OpenMP).
int orc_threads(void) {
#ifdef _OPENMP
  int n = 1;
#pragma omp parallel
  {
#pragma omp single
    n = omp_get_num_threads();
  }
  return n;
#else
  return 1;
#endif
}

// Applies single actions, for tests: op = 0 potential, 1 kinetic.
int orc_action(const orc_problem* prob, int op, double tau, double* psi_io) {
  Grid g;
  if (!make_grid(prob, g) || !prob->vtable) return -1;
  cd* psi = reinterpret_cast<cd*>(psi_io);
  if (op == 0) {
    PotentialEigen pe;
    potential_eigen(g, prob->vtable, pe);
    potential_action(g, pe, tau, psi);
  } else {
    kinetic_action(g, tau, psi);
  }
  return 0;
}

// ---------------------------------------------------------------- observables
// out[0] = norm <psi|psi>, out[1] = energy <psi|H|psi>, out[2+s] = population
// of surface s, out[2+S] = <T>, out[3+S] = <V>.  Inner products carry the
// volume element dV (Sec. "Geometric properties of the exact evolution
// operator": norm, energy).  <T> is evaluated in the momentum representation
// with Parseval's factor 1/N_g; <V> pointwise.
int orc_observables(const orc_problem* prob, const double* psi_in, double* out) {
  Grid g;
  if (!make_grid(prob, g) || !prob->vtable) return -1;
  const int S = g.S;
  const cd* psi = reinterpret_cast<const cd*>(psi_in);
  // Sums over up to ~1e7 grid points accumulate in long double so that the
  // reduction itself stays far below the 1e-12 invariant errors of interest.
  std::vector<double> pop(S, 0.0);
  for (int s = 0; s < S; ++s) {
    ld acc = 0;
    for (int64_t x = 0; x < g.npts; ++x) acc += (ld)std::norm(psi[s * g.npts + x]);
    pop[s] = (double)(acc * (ld)g.dV);
  }
  ld evl = 0;
  for (int64_t x = 0; x < g.npts; ++x) {
    for (int i = 0; i < S; ++i)
      for (int j = 0; j < S; ++j) {
        double v = prob->vtable[(int64_t)packed_index(S, i, j) * g.npts + x];
        evl += (ld)(std::conj(psi[i * g.npts + x]) * v * psi[j * g.npts + x]).real();
      }
  }
  const double ev = (double)(evl * (ld)g.dV);
  std::vector<cd> tmp(psi, psi + (size_t)S * g.npts);
  fft_state(g, tmp.data(), false);
  ld etl = 0;
  for (int64_t k = 0; k < g.npts; ++k) {
    double t = kinetic_energy_at(g, k);
    for (int s = 0; s < S; ++s) etl += (ld)(t * std::norm(tmp[s * g.npts + k]));
  }
  const double et = (double)(etl * (ld)g.dV / (ld)g.npts);
  ld norm = 0;
  for (int s = 0; s < S; ++s) norm += (ld)pop[s];
  out[0] = (double)norm;
  out[1] = et + ev;
  for (int s = 0; s < S; ++s) out[2 + s] = pop[s];
  out[2 + S] = et;
  out[3 + S] = ev;
  return 0;
}

// <psi|phi> with the volume element (Sec. "Geometric properties ...").
int orc_overlap(const orc_problem* prob, const double* psi_in, const double* phi_in,
                double* out) {
  Grid g;
  if (!make_grid(prob, g)) return -1;
  const cd* psi = reinterpret_cast<const cd*>(psi_in);
  const cd* phi = reinterpret_cast<const cd*>(phi_in);
  ld re = 0, im = 0;
  for (int64_t i = 0; i < (int64_t)g.S * g.npts; ++i) {
    cd z = std::conj(psi[i]) * phi[i];
    re += (ld)z.real();
    im += (ld)z.imag();
  }
  out[0] = (double)(re * (ld)g.dV);
  out[1] = (double)(im * (ld)g.dV);
  return 0;
}

// L2 distance ||psi - phi|| = sqrt(sum |psi - phi|^2 dV), the error norm of
// the convergence studies (Sec. "Numerical examples"), from the difference
// itself: the expansion ||psi||^2 + ||phi||^2 - 2 Re<psi|phi> cancels
// catastrophically when the two states agree closely.
int orc_distance(const orc_problem* prob, const double* psi_in, const double* phi_in,
                 double* out) {
  Grid g;
  if (!make_grid(prob, g)) return -1;
  const cd* psi = reinterpret_cast<const cd*>(psi_in);
  const cd* phi = reinterpret_cast<const cd*>(phi_in);
  ld d2 = 0;
  for (int64_t i = 0; i < (int64_t)g.S * g.npts; ++i) d2 += (ld)std::norm(psi[i] - phi[i]);
  out[0] = (double)std::sqrt(d2 * (ld)g.dV);
  return 0;
}

// ---------------------------------------------------------------- brute force
// Exact evolution exp(-i H t / hbar) psi for the discrete Hamiltonian on
// tiny grids (Eq. exact_evol_op): H = K (x) 1_S + blockdiag V(x), where the
// kinetic matrix of each axis is the circulant (1/n) sum_k T(p_k) cos(2 pi k
// (j-l)/n) (real because T is even in p).  H is diagonalised by the Jacobi
// solver and psi(t) = R exp(-i Lambda t/hbar) R^T psi(0).  Returns -1 when
// S * npts exceeds 512.
int orc_exact(const orc_problem* prob, double t, double* psi_io) {
  Grid g;
  if (!make_grid(prob, g) || !prob->vtable) return -1;
  const int64_t dim = (int64_t)g.S * g.npts;
  if (dim > 512) return -1;
  const int n = (int)dim;
  std::vector<double> H((size_t)n * n, 0.0);
  auto idx = [&](int s, int64_t x) { return (int)(s * g.npts + x); };
  // kinetic part
  for (int d = 0; d < g.ndim; ++d) {
    const int nd = g.n[d];
    std::vector<double> Kd((size_t)nd * nd, 0.0);
    for (int j = 0; j < nd; ++j)
      for (int l = 0; l < nd; ++l) {
        ld acc = 0;
        for (int k = 0; k < nd; ++k) {
          double p = momentum(g, d, k);
          ld tk = 0.5L * (ld)g.inv_mass[d] * (ld)p * (ld)p;
          int m = ((j - l) % nd + nd) % nd;
          acc += tk * cosl(2.0L * PI_L * (ld)k * (ld)m / (ld)nd);
        }
        Kd[(size_t)j * nd + l] = (double)(acc / (ld)nd);
      }
    for (int64_t x = 0; x < g.npts; ++x) {
      int jd = (int)((x / g.stride[d]) % nd);
      for (int l = 0; l < nd; ++l) {
        int64_t y = x + (int64_t)(l - jd) * g.stride[d];
        for (int s = 0; s < g.S; ++s) H[(size_t)idx(s, x) * n + idx(s, y)] += Kd[(size_t)jd * nd + l];
      }
    }
  }
  // potential part
  for (int64_t x = 0; x < g.npts; ++x)
    for (int i = 0; i < g.S; ++i)
      for (int j = 0; j < g.S; ++j)
        H[(size_t)idx(i, x) * n + idx(j, x)] +=
            prob->vtable[(int64_t)packed_index(g.S, i, j) * g.npts + x];
  std::vector<double> R, lam;
  jacobi_eigen(n, H, R, lam);
  cd* psi = reinterpret_cast<cd*>(psi_io);
  std::vector<cd> c(n, cd(0, 0)), out(n, cd(0, 0));
  for (int l = 0; l < n; ++l) {
    cd acc(0, 0);
    for (int r = 0; r < n; ++r) acc += R[(size_t)r * n + l] * psi[r];
    double ph = -lam[l] * t / g.hbar;
    c[l] = acc * cd(std::cos(ph), std::sin(ph));
  }
  for (int r = 0; r < n; ++r) {
    cd acc(0, 0);
    for (int l = 0; l < n; ++l) acc += R[(size_t)r * n + l] * c[l];
    out[r] = acc;
  }
  std::copy(out.begin(), out.end(), psi);
  return 0;
}

}  // extern "C"

// ---------------------------------------------------------------- gradients
// Derivatives of surface populations with respect to parameters theta_k of
// a potential linear in them, V(theta) = V + sum_k theta_k D_k, by forward
// (tangent) propagation of d psi / d theta_k alongside psi.  Kinetic actions
// do not depend on theta; a potential action psi <- U psi with
// U = exp(-i tau V / hbar) gives d psi <- U d psi + L_k psi, where L_k is the
// Frechet derivative of the exponential in direction D_k, read off the
// upper-right block of exp([[A, E], [0, A]]) with A = -i tau V / hbar,
// E = -i tau D_k / hbar.  That block exponential is evaluated in long double
// by scaling and squaring of its Taylor series.

typedef std::complex<ld> cl;

// exp(M) for an n x n complex matrix (row-major), scaling and squaring.
static void expm_taylor(int n, const std::vector<cl>& M, std::vector<cl>& out) {
  ld norm = 0;
  for (int i = 0; i < n; ++i) {
    ld row = 0;
    for (int j = 0; j < n; ++j) row += std::abs(M[(size_t)i * n + j]);
    norm = std::max(norm, row);
  }
  int sq = 0;
  while (norm > 0.25L) {
    norm /= 2;
    ++sq;
  }
  const ld scale = std::ldexp(1.0L, -sq);
  std::vector<cl> A(M), term((size_t)n * n), next((size_t)n * n);
  for (auto& a : A) a *= scale;
  out.assign((size_t)n * n, cl(0, 0));
  for (int i = 0; i < n; ++i) out[(size_t)i * n + i] = 1;
  term = out;  // identity
  for (int k = 1; k <= 30; ++k) {
    for (int i = 0; i < n; ++i)
      for (int j = 0; j < n; ++j) {
        cl acc(0, 0);
        for (int l = 0; l < n; ++l) acc += term[(size_t)i * n + l] * A[(size_t)l * n + j];
        next[(size_t)i * n + j] = acc / (ld)k;
      }
    term.swap(next);
    for (size_t q = 0; q < out.size(); ++q) out[q] += term[q];
  }
  for (int r = 0; r < sq; ++r) {
    for (int i = 0; i < n; ++i)
      for (int j = 0; j < n; ++j) {
        cl acc(0, 0);
        for (int l = 0; l < n; ++l) acc += out[(size_t)i * n + l] * out[(size_t)l * n + j];
        next[(size_t)i * n + j] = acc;
      }
    out.swap(next);
  }
}

// U = exp(-i tau V/hbar) and L = its Frechet derivative in direction D, both
// S x S complex (double), from the 2S x 2S block exponential.
static void expm_frechet_point(int S, const double* V, const double* D, double tau, double hbar,
                               cd* U, cd* L) {
  const int n = 2 * S;
  std::vector<cl> M((size_t)n * n, cl(0, 0)), E;
  const cl f(0, -(ld)tau / (ld)hbar);
  for (int i = 0; i < S; ++i)
    for (int j = 0; j < S; ++j) {
      M[(size_t)i * n + j] = f * (ld)V[i * S + j];
      M[(size_t)(i + S) * n + (j + S)] = f * (ld)V[i * S + j];
      M[(size_t)i * n + (j + S)] = f * (ld)D[i * S + j];
    }
  expm_taylor(n, M, E);
  for (int i = 0; i < S; ++i)
    for (int j = 0; j < S; ++j) {
      if (U) U[i * S + j] = cd((double)E[(size_t)i * n + j].real(), (double)E[(size_t)i * n + j].imag());
      if (L)
        L[i * S + j] = cd((double)E[(size_t)i * n + j + S].real(), (double)E[(size_t)i * n + j + S].imag());
    }
}

static void unpack_matrix(int S, const double* table, int64_t npts, int64_t x, double* M) {
  for (int i = 0; i < S; ++i)
    for (int j = 0; j < S; ++j) M[i * S + j] = table[(int64_t)packed_index(S, i, j) * npts + x];
}

extern "C" {

// Frechet derivative of exp(-i tau V / hbar) in direction D (real symmetric
// S x S, row-major); U and L receive S x S complex (interleaved).
int orc_expm_frechet(int S, const double* V, const double* D, double tau, double hbar, double* U,
                     double* L) {
  if (S < 1 || S > 16) return -1;
  expm_frechet_point(S, V, D, tau, hbar, reinterpret_cast<cd*>(U), reinterpret_cast<cd*>(L));
  return 0;
}

// Populations P_s(T) of psi propagated nsteps steps (pruned sequence) and
// grad[k] = sum_s weights[s] dP_s/dtheta_k, by tangent propagation.
// dvtables: [nparams][S(S+1)/2][npts] packed like the V-table.
// pops: [S] out; grad: [nparams] out.  Returns 0 or -1.
int orc_gradient(const orc_problem* prob, int nparams, const double* dvtables, int split,
                 int scheme, int order, double dt, int64_t nsteps, const double* psi0,
                 const double* weights, double* pops, double* grad) {
  Grid g;
  if (!make_grid(prob, g) || !prob->vtable || nparams < 0 || nsteps < 0) return -1;
  std::vector<ld> la, lb;
  if (!splitting_ld(split, scheme, order, true, la, lb)) return -1;
  std::vector<double> a(la.begin(), la.end()), b(lb.begin(), lb.end());
  const int S = g.S;
  const int64_t n = (int64_t)S * g.npts;
  std::vector<cd> psi(reinterpret_cast<const cd*>(psi0), reinterpret_cast<const cd*>(psi0) + n);
  std::vector<std::vector<cd>> dpsi(nparams, std::vector<cd>(n, cd(0, 0)));
  const bool aV = a_is_potential(split);

  auto potential = [&](double tau) {
#pragma omp parallel
    {
      std::vector<double> V((size_t)S * S), D((size_t)S * S);
      std::vector<cd> U((size_t)S * S), L((size_t)S * S), v(S), w(S);
#pragma omp for schedule(static)
      for (int64_t x = 0; x < g.npts; ++x) {
        unpack_matrix(S, prob->vtable, g.npts, x, V.data());
        for (int s = 0; s < S; ++s) v[s] = psi[s * g.npts + x];
        for (int k = 0; k < nparams; ++k) {
          unpack_matrix(S, dvtables + (int64_t)k * (S * (S + 1) / 2) * g.npts, g.npts, x, D.data());
          expm_frechet_point(S, V.data(), D.data(), tau, g.hbar, U.data(), L.data());
          for (int i = 0; i < S; ++i) {
            cd acc(0, 0);
            for (int j = 0; j < S; ++j)
              acc += U[i * S + j] * dpsi[k][j * g.npts + x] + L[i * S + j] * v[j];
            w[i] = acc;
          }
          for (int s = 0; s < S; ++s) dpsi[k][s * g.npts + x] = w[s];
        }
        if (nparams == 0) {
          std::vector<double> Z((size_t)S * S, 0.0);
          expm_frechet_point(S, V.data(), Z.data(), tau, g.hbar, U.data(), nullptr);
        }
        for (int i = 0; i < S; ++i) {
          cd acc(0, 0);
          for (int j = 0; j < S; ++j) acc += U[i * S + j] * v[j];
          psi[i * g.npts + x] = acc;
        }
      }
    }
  };
  auto kinetic = [&](double tau) {
    kinetic_action(g, tau, psi.data());
    for (int k = 0; k < nparams; ++k) kinetic_action(g, tau, dpsi[k].data());
  };
  for (int64_t step = 0; step < nsteps; ++step) {
    for (size_t j = 0; j < a.size(); ++j) {
      if (aV) potential(a[j] * dt); else kinetic(a[j] * dt);
      if (b[j] != 0.0) {
        if (aV) kinetic(b[j] * dt); else potential(b[j] * dt);
      }
    }
  }
  for (int s = 0; s < S; ++s) {
    ld acc = 0;
    for (int64_t x = 0; x < g.npts; ++x) acc += (ld)std::norm(psi[s * g.npts + x]);
    pops[s] = (double)(acc * (ld)g.dV);
  }
  for (int k = 0; k < nparams; ++k) {
    ld acc = 0;
    for (int s = 0; s < S; ++s)
      for (int64_t x = 0; x < g.npts; ++x) {
        const cd z = std::conj(psi[s * g.npts + x]) * dpsi[k][s * g.npts + x];
        acc += (ld)weights[s] * 2.0L * (ld)z.real();
      }
    grad[k] = (double)(acc * (ld)g.dV);
  }
  return 0;
}

}  // extern "C"
