// kernels_3d.hip -- three-dimensional cubic grids n^3: the composed time step
// as a sequence of pencil passes over psi[s][z][y][x] (x fastest).
//
// A substep (one potential action followed by one kinetic action, Sec.
// "Dynamic Fourier method") is four passes over the state:
//   z-pass : [inverse FFT along z] -> potential unitary(ies) -> [forward FFT z]
//            (all S surfaces of a tile of x-columns, so the S x S matvec of
//            Sec. "Molecular Hamiltonian in the diabatic basis" runs in
//            registers);
//   y-pass : forward FFT along y;
//   x-pass : forward FFT along x -> kinetic phase -> inverse FFT along x;
//   y-pass : inverse FFT along y.
// Between passes the z axis stays in the momentum representation, so the
// potential's own pass carries the z transforms.  The last potential action
// of a step and the first of the next share one z-pass (two matvecs in
// registers; the arithmetic is the same as two separate passes).
// The kinetic factor is separable, exp(-i tau T(p)/hbar) / (n_y n_x) =
// f_z(k_z) f_y(k_y) f_x(k_x); the planner stores the three per-axis factors
// of each unique coefficient.  The 1/n_z of the z round trip is applied by
// the z-pass after its inverse transform, because consecutive kinetic
// actions (TVT at a step boundary) share one z round trip.
#include <type_traits>
#include <vector>

#include "passes_3d.hpp"

namespace sop {
namespace {

using namespace s3d;

// Schedules of the adjoint z-pass (2S pencils per thread): four values per
// thread and pencil.
template <class SC>
struct AdjSched;
template <>
struct AdjSched<Z32> {
  using type = Sched<32, 4, RList<4, 4, 2>, RList<2, 4, 4>, 4, 2>;
};
template <>
struct AdjSched<Z64> {
  using type = Sched<64, 4, RList<4, 4, 4>, RList<4, 4, 4>, 4, 4>;
};
template <>
struct AdjSched<Z128> {
  using type = Sched<128, 4, RList<4, 4, 4, 2>, RList<2, 4, 4, 4>, 4, 2>;
};
template <>
struct AdjSched<Z256> {
  using type = Sched<256, 4, RList<4, 4, 4, 4>, RList<4, 4, 4, 4>, 4, 4>;
};

// Columns per tile of the z-pass: the table tile width.
template <class SC, typename T>
constexpr int zcols() {
  return kTableCols;
}

// ---------------------------------------------------------------- z-pass
template <typename T, class SC, int S, int C, bool PRE_INV, bool POST_FWD>
__global__ void __launch_bounds__(C * SC::TPC)
    k3d_zpass(cx<T>* __restrict__ psi, const cx<T>* __restrict__ vexp, int nv, int iv0, int iv1,
              int conj, const cx<T>* __restrict__ tw) {
  extern __shared__ char smem_raw[];
  cx<T>* lds = reinterpret_cast<cx<T>*>(smem_raw);
  psi += (size_t)blockIdx.z * S * ((size_t)SC::N * SC::N * SC::N);  // member of a batch
  zpass_body<T, SC, S, C, C, PRE_INV, POST_FWD>(psi, vexp, nv, iv0, iv1, conj, tw, lds,
                                                blockIdx.x, blockIdx.y);
}

// ---------------------------------------------------------------- adjoint z-pass
// Backward sweep of the adjoint method over the stacked state [psi; lambda]
// (2S pencils, FP64).  For each potential action j, walked in reverse, the
// kernel holds psi_j (the state after the action) and lambda_j (the adjoint
// after it) and computes
//   psi_{j-1} = U_j^dag psi_j,   lambda_{j-1} = U_j^dag lambda_j,
//   Q(x) += R Re(M) R^T,  M_ab = conj(alpha_a) F_ab beta_b,
// with alpha = R^T lambda_j, beta = R^T psi_{j-1}, V(x) = R diag(lam) R^T and
// the divided differences of f(v) = exp(-i tau v):
//   F_ab = (f(lam_a) - f(lam_b)) / (lam_a - lam_b)
//        = -i tau exp(-i tau (lam_a + lam_b)/2) sinc(tau (lam_a - lam_b)/2),
// so that d P / d theta_k = 2 dV sum_x sum_ij Q_ij(x) D_k,ij(x) (Daleckii-
// Krein form of the Frechet derivative of exp(-i tau V(theta))).  Q is kept
// packed (Q_ii; Q_ij + Q_ji for i < j) in qacc[entry][point].
template <class SC, int S, int C, bool PRE_INV, bool POST_FWD>
__global__ void __launch_bounds__(C * SC::TPC)
    k3d_zpass_adj(cx<double>* __restrict__ stk, const cx<double>* __restrict__ vexp,
                  const cx<double>* __restrict__ eig, double* __restrict__ qacc,
                  const double* __restrict__ taus, int nv, int iv0, int iv1,
                  const cx<double>* __restrict__ tw) {
  extern __shared__ char smem_raw[];
  cx<double>* lds = reinterpret_cast<cx<double>*>(smem_raw);
  constexpr int N = SC::N, E = SC::E, NE = S * (S + 1) / 2, P = 2 * S;
  const int lane = threadIdx.x;
  const int col = lane % C, t = lane / C;
  const int x = blockIdx.x * C + col, y = blockIdx.y;
  constexpr uint32_t plane = (uint32_t)N * N;
  constexpr int64_t npts = (int64_t)plane * N;
  constexpr uint32_t tile = (uint32_t)N * NE * C;
  const uint32_t off0 = (uint32_t)y * N + x;
  const size_t tbase = ((size_t)y * (N / C) + blockIdx.x) * tile;
  const LayStrided lay{col, 0, C};
  cx<double> v[P][E];
  constexpr int RIN = PRE_INV ? SC::RL : SC::RF;
#pragma unroll
  for (int s = 0; s < P; ++s) {
    const auto rs = rsrc(stk + s * npts, (uint32_t)npts);
#pragma unroll
    for (int q = 0; q < E; ++q) v[s][q] = ld<double>(rs, own_idx<N, E, RIN>(t, q) * plane + off0);
  }
  if constexpr (PRE_INV) {
#pragma unroll
    for (int s = 0; s < P; ++s) fft_inverse<SC, 1>(v + s, lds, lay, tw, t);
    constexpr double inv_n = 1.0 / (double)N;
#pragma unroll
    for (int s = 0; s < P; ++s)
#pragma unroll
      for (int q = 0; q < E; ++q) v[s][q] = cx<double>{v[s][q].re * inv_n, v[s][q].im * inv_n};
  }
  auto vact = [&](int iv) {
    const auto ru = rsrc(vexp + (size_t)iv * NE * npts + tbase, tile);
    const auto rg = rsrc(eig + tbase, tile);
    const double tau = taus[iv];
#pragma unroll
    for (int q = 0; q < E; ++q) {
      const uint32_t tp = (uint32_t)own_idx<N, E, SC::RF>(t, q) * (NE * C) + col;
      const uint32_t pt = (uint32_t)own_idx<N, E, SC::RF>(t, q) * plane + off0;
      cx<double> u[NE];
#pragma unroll
      for (int e = 0; e < NE; ++e) {
        u[e] = ld<double>(ru, tp + e * C);
        u[e].im = -u[e].im;  // U^dag = conj(U) for complex-symmetric U
      }
      double ev[2 * NE];  // R (row-major S x S) then lam (S)
#pragma unroll
      for (int e = 0; e < NE; ++e) {
        const cx<double> w = ld<double>(rg, tp + e * C);
        ev[2 * e] = w.re;
        ev[2 * e + 1] = w.im;
      }
      cx<double> ps[S], la[S];
#pragma unroll
      for (int s = 0; s < S; ++s) {
        ps[s] = v[s][q];
        la[s] = v[S + s][q];
      }
      apply_u<double, S>(ps, u);  // psi_{j-1}
      // alpha = R^T lambda_j, beta = R^T psi_{j-1}
      cx<double> al[S], be[S];
#pragma unroll
      for (int a = 0; a < S; ++a) {
        al[a] = cx<double>{0.0, 0.0};
        be[a] = cx<double>{0.0, 0.0};
#pragma unroll
        for (int i = 0; i < S; ++i) {
          const double r = ev[i * S + a];
          al[a] = cx<double>{al[a].re + r * la[i].re, al[a].im + r * la[i].im};
          be[a] = cx<double>{be[a].re + r * ps[i].re, be[a].im + r * ps[i].im};
        }
      }
      const double* lam = ev + S * S;
      double rm[S][S];  // Re(M)
#pragma unroll
      for (int a = 0; a < S; ++a)
#pragma unroll
        for (int b = 0; b < S; ++b) {
          // F_ab = -i tau exp(-i tau (lam_a + lam_b)/2) sinc(tau (lam_a - lam_b)/2)
          const double h = 0.5 * tau * (lam[a] - lam[b]);
          const double sc = (fabs(h) < 1e-8) ? 1.0 - h * h / 6.0 : sin(h) / h;
          double sn, cs;
          sincos(-0.5 * tau * (lam[a] + lam[b]), &sn, &cs);
          // -i tau (cs + i sn) sc = tau sc (sn - i cs)
          const cx<double> F = {tau * sc * sn, -tau * sc * cs};
          const cx<double> fb = cmul(F, be[b]);
          rm[a][b] = al[a].re * fb.re + al[a].im * fb.im;  // Re(conj(alpha_a) F_ab beta_b)
        }
      // Q = R Re(M) R^T, accumulated packed
      int e = 0;
#pragma unroll
      for (int i = 0; i < S; ++i)
#pragma unroll
        for (int j = i; j < S; ++j) {
          double qij = 0.0, qji = 0.0;
#pragma unroll
          for (int a = 0; a < S; ++a)
#pragma unroll
            for (int b = 0; b < S; ++b) {
              qij += ev[i * S + a] * rm[a][b] * ev[j * S + b];
              qji += ev[j * S + a] * rm[a][b] * ev[i * S + b];
            }
          double* qp = qacc + (size_t)e * npts + pt;
          *qp += (i == j) ? qij : qij + qji;
          ++e;
        }
      apply_u<double, S>(la, u);  // lambda_{j-1}
#pragma unroll
      for (int s = 0; s < S; ++s) {
        v[s][q] = ps[s];
        v[S + s][q] = la[s];
      }
    }
  };
  if (nv >= 1) vact(iv0);
  if (nv >= 2) vact(iv1);
  if constexpr (POST_FWD) {
#pragma unroll
    for (int s = 0; s < P; ++s) fft_forward<SC, 1>(v + s, lds, lay, tw, t);
  }
  constexpr int ROUT = POST_FWD ? SC::RL : SC::RF;
#pragma unroll
  for (int s = 0; s < P; ++s) {
    const auto rs = rsrc(stk + s * npts, (uint32_t)npts);
#pragma unroll
    for (int q = 0; q < E; ++q) st(rs, own_idx<N, E, ROUT>(t, q) * plane + off0, v[s][q]);
  }
}

// ---------------------------------------------------------------- y-pass
// grid (N / C, N, surfaces x states): blockIdx.z picks one surface pencil set
template <typename T, class SC, int C, bool INV>
__global__ void __launch_bounds__(C * SC::TPC)
    k3d_ypass(cx<T>* __restrict__ psi, const cx<T>* __restrict__ tw) {
  extern __shared__ char smem_raw[];
  cx<T>* lds = reinterpret_cast<cx<T>*>(smem_raw);
  constexpr int64_t npts = (int64_t)SC::N * SC::N * SC::N;
  ypass_body<T, SC, C, INV>(psi + blockIdx.z * npts, tw, lds, blockIdx.x, blockIdx.y);
}

// ---------------------------------------------------------------- x-pass
template <typename T, class SC, int ROWS, int MODE>
__global__ void __launch_bounds__(ROWS * SC::TPC)
    k3d_xpass(cx<T>* __restrict__ psi, const cx<T>* __restrict__ tw,
              const cx<T>* __restrict__ kin, int conj) {
  extern __shared__ char smem_raw[];
  cx<T>* lds = reinterpret_cast<cx<T>*>(smem_raw);
  constexpr int64_t npts = (int64_t)SC::N * SC::N * SC::N;
  xpass_body<T, SC, ROWS, MODE>(psi + blockIdx.z * npts, tw, kin, conj, lds, blockIdx.x,
                                blockIdx.y);
}

// ---------------------------------------------------------------- xy plane
// grid (N planes, surfaces x states)
template <typename T, class SC>
__global__ void __launch_bounds__(SC::N * SC::TPC)
    k3d_plane(cx<T>* __restrict__ psi, const cx<T>* __restrict__ tw,
              const cx<T>* __restrict__ kin, int conj) {
  extern __shared__ char smem_raw[];
  cx<T>* lds = reinterpret_cast<cx<T>*>(smem_raw);
  constexpr int64_t npts = (int64_t)SC::N * SC::N * SC::N;
  plane_body<T, SC>(psi + blockIdx.y * npts, tw, kin, conj, lds, blockIdx.x);
}

// ---------------------------------------------------------------- launchers
// Pass program of the 3D executor.  The machine walks the step program:
// a potential action opens (or joins, up to two) a z-pass that inverts the
// z transform first when the state is z-transformed; a kinetic action closes
// the open z-pass with a forward z transform (or adds a transform-only
// z-pass) and adds y-forward, x (phase), y-inverse.
struct PassMachine {
  bool zk = false, zopen = false, zpre = false;
  int zv[2] = {0, 0}, znv = 0;
  bool operator==(const PassMachine& o) const {
    return zk == o.zk && zopen == o.zopen && zpre == o.zpre && znv == o.znv &&
           (znv < 1 || zv[0] == o.zv[0]) && (znv < 2 || zv[1] == o.zv[1]);
  }
};

void flush_z(PassMachine& m, bool post_fwd, std::vector<PassDesc>& out) {
  PassDesc p;
  p.kind = PassDesc::Z;
  p.pre_inv = m.zpre;
  p.post_fwd = post_fwd;
  p.nv = m.znv;
  p.iv0 = m.zv[0];
  p.iv1 = m.zv[1];
  out.push_back(p);
  m.zopen = false;
  m.znv = 0;
  m.zk = post_fwd;
}

void emit_step(const DevView& d, PassMachine& m, std::vector<PassDesc>& out, bool xy) {
  for (int a = 0; a < d.nact; ++a) {
    const int code = d.hprog[a];
    const int idx = prog_idx(code);
    if (prog_op(code) == OP_V) {
      if (m.zopen && m.znv == 2) flush_z(m, false, out);
      if (!m.zopen) {
        m.zopen = true;
        m.zpre = m.zk;
        m.znv = 0;
        m.zk = false;
      }
      m.zv[m.znv++] = idx;
    } else {
      if (m.zopen) {
        flush_z(m, true, out);
      } else if (!m.zk) {
        PassDesc p;
        p.kind = PassDesc::Z;
        p.post_fwd = true;
        out.push_back(p);
        m.zk = true;
      }
      if (xy) {
        PassDesc p;
        p.kind = PassDesc::XY;
        p.tidx = idx;
        out.push_back(p);
        continue;
      }
      PassDesc y, x, yi;
      y.kind = PassDesc::YF;
      x.kind = PassDesc::XP;
      x.tidx = idx;
      yi.kind = PassDesc::YI;
      out.push_back(y);
      out.push_back(x);
      out.push_back(yi);
    }
  }
}

void emit_flush(PassMachine& m, std::vector<PassDesc>& out) {
  if (m.zopen) {
    flush_z(m, false, out);
  } else if (m.zk) {
    PassDesc p;
    p.kind = PassDesc::Z;
    p.pre_inv = true;
    out.push_back(p);
    m.zk = false;
  }
}

template <typename K>
hipError_t set_lds(K k, size_t bytes) {
  if (bytes <= 64 * 1024) return hipSuccess;
  return hipFuncSetAttribute((const void*)k, hipFuncAttributeMaxDynamicSharedMemorySize,
                             (int)bytes);
}

template <typename T, class SC, int S>
struct Passes {
  static constexpr int N = SC::N;
  using XS = typename XYSched<SC>::type;
  static constexpr int C = cols<XS, T>();
  static constexpr int CZ = zcols<SC, T>();
  static constexpr int ROWS = xrows<XS>();
  static_assert(N % C == 0 && N % CZ == 0 && N % ROWS == 0, "tiles must cover the grid");

  // algorithmic bytes of one pass: psi read + written, plus tables read
  static double pass_bytes(const DevView& d, int ntables) {
    return (2.0 * S + ntables * S * (S + 1) / 2.0) * (double)d.npts * sizeof(cx<T>) * d.count;
  }

  template <bool PI, bool PF>
  static hipError_t z(const DevView& d, cx<T>* psi, int nv, int iv0, int iv1, int conj) {
    auto k = k3d_zpass<T, SC, S, CZ, PI, PF>;
    const size_t lds = (size_t)CZ * N * sizeof(cx<T>);
    hipError_t e = set_lds(k, lds);
    if (e != hipSuccess) return e;
    TimedLaunch tl(d, KIND_ZPASS, pass_bytes(d, nv));
    hipLaunchKernelGGL(k, dim3(N / CZ, N, d.count), dim3(CZ * SC::TPC), lds, d.stream, psi,
                       (const cx<T>*)d.vexp, nv, iv0, iv1, conj, (const cx<T>*)d.tw[0]);
    return hipGetLastError();
  }
  static hipError_t zpass(const DevView& d, cx<T>* psi, bool pi, bool pf, int nv, int iv0,
                          int iv1, int conj) {
    if (pi && pf) return z<true, true>(d, psi, nv, iv0, iv1, conj);
    if (pi) return z<true, false>(d, psi, nv, iv0, iv1, conj);
    if (pf) return z<false, true>(d, psi, nv, iv0, iv1, conj);
    return z<false, false>(d, psi, nv, iv0, iv1, conj);
  }
  template <bool INV>
  static hipError_t ypass(const DevView& d, cx<T>* psi) {
    auto k = k3d_ypass<T, XS, C, INV>;
    const size_t lds = (size_t)C * N * sizeof(cx<T>);
    hipError_t e = set_lds(k, lds);
    if (e != hipSuccess) return e;
    TimedLaunch tl(d, KIND_YPASS, pass_bytes(d, 0));
    hipLaunchKernelGGL(k, dim3(N / C, N, d.S * d.count), dim3(C * XS::TPC), lds, d.stream, psi,
                       (const cx<T>*)d.tw[1]);
    return hipGetLastError();
  }
  template <int MODE>
  static hipError_t xpass(const DevView& d, cx<T>* psi, int tidx, int conj) {
    auto k = k3d_xpass<T, XS, ROWS, MODE>;
    const size_t lds = (size_t)ROWS * (N + N / 16) * sizeof(cx<T>);
    hipError_t e = set_lds(k, lds);
    if (e != hipSuccess) return e;
    const cx<T>* kin = (const cx<T>*)d.kin + (size_t)tidx * 3 * d.kin_stride;
    TimedLaunch tl(d, KIND_XPASS, pass_bytes(d, 0));
    hipLaunchKernelGGL(k, dim3(N / ROWS, N, d.S * d.count), dim3(ROWS * XS::TPC), lds, d.stream, psi,
                       (const cx<T>*)d.tw[2], kin, conj);
    return hipGetLastError();
  }

  static constexpr bool PLANE = plane_fits<T, XS>();
  static hipError_t plane(const DevView& d, cx<T>* psi, int tidx, int conj) {
    if constexpr (!PLANE) {
      return hipErrorInvalidValue;
    } else {
      auto k = k3d_plane<T, XS>;
      const size_t lds = plane_lds_elems<T, XS>() * sizeof(cx<T>);
      hipError_t e = set_lds(k, lds);
      if (e != hipSuccess) return e;
      const cx<T>* kin = (const cx<T>*)d.kin + (size_t)tidx * 3 * d.kin_stride;
      TimedLaunch tl(d, KIND_PLANE, pass_bytes(d, 0));
      hipLaunchKernelGGL(k, dim3(N, d.S * d.count), dim3(N * XS::TPC), lds, d.stream, psi,
                         (const cx<T>*)d.tw[0], kin, conj);
      return hipGetLastError();
    }
  }

  // Launches one pass descriptor.
  static hipError_t launch(const DevView& d, cx<T>* psi, const PassDesc& p, int conj) {
    switch (p.kind) {
      case PassDesc::Z: return zpass(d, psi, p.pre_inv, p.post_fwd, p.nv, p.iv0, p.iv1, conj);
      case PassDesc::YF: return ypass<false>(d, psi);
      case PassDesc::YI: return ypass<true>(d, psi);
      case PassDesc::XY: return plane(d, psi, p.tidx, conj);
      default: return xpass<XP_PHASE>(d, psi, p.tidx, conj);
    }
  }
  static hipError_t launch_all(const DevView& d, cx<T>* psi, const std::vector<PassDesc>& v,
                               int conj) {
    for (const PassDesc& p : v) {
      hipError_t e = launch(d, psi, p, conj);
      if (e != hipSuccess) return e;
    }
    return hipSuccess;
  }

  static hipError_t propagate(const DevView& d, void* vpsi, int64_t nsteps, int conj) {
    cx<T>* psi = (cx<T>*)vpsi;
    const bool xy = PLANE && d.plane;
    PassMachine m0;
    std::vector<PassDesc> first, body, tail;
    PassMachine m1 = m0;
    emit_step(d, m1, first, xy);
    const bool use_graph = d.graphs != nullptr && d.timer == nullptr && nsteps >= 4;
    if (!use_graph) {
      hipError_t e = launch_all(d, psi, first, conj);
      if (e != hipSuccess) return e;
      PassMachine m = m1;
      for (int64_t step = 1; step < nsteps; ++step) {
        body.clear();
        emit_step(d, m, body, xy);
        if ((e = launch_all(d, psi, body, conj)) != hipSuccess) return e;
      }
      emit_flush(m, tail);
      return launch_all(d, psi, tail, conj);
    }
    PassMachine m2 = m1;
    emit_step(d, m2, body, xy);
    PassMachine m3 = m2;
    std::vector<PassDesc> body2;
    emit_step(d, m3, body2, xy);
    if (!(m2 == m3) || !(body == body2)) {  // no steady state: launch eagerly
      DevView e = d;
      e.graphs = nullptr;
      return propagate(e, vpsi, nsteps, conj);
    }
    emit_flush(m2, tail);
    // graphs keyed by (state pointer, direction, member count, segment)
    auto seg = [&](int which, const std::vector<PassDesc>& v, hipGraphExec_t* out) -> hipError_t {
      GraphCache::Key key{(const void*)psi, conj, d.count, which};
      auto it = d.graphs->execs.find(key);
      if (it != d.graphs->execs.end()) {
        *out = it->second;
        return hipSuccess;
      }
      DevView c = d;
      c.stream = d.graphs->capture;
      hipError_t e = hipStreamBeginCapture(c.stream, hipStreamCaptureModeThreadLocal);
      if (e != hipSuccess) return e;
      hipError_t le = launch_all(c, psi, v, conj);
      hipGraph_t g = nullptr;
      e = hipStreamEndCapture(c.stream, &g);
      if (le != hipSuccess) {
        if (g) (void)hipGraphDestroy(g);
        return le;
      }
      if (e != hipSuccess) return e;
      hipGraphExec_t x = nullptr;
      e = hipGraphInstantiate(&x, g, nullptr, nullptr, 0);
      (void)hipGraphDestroy(g);
      if (e != hipSuccess) return e;
      d.graphs->execs[key] = x;
      *out = x;
      return hipSuccess;
    };
    hipGraphExec_t g1, g2, g3;
    hipError_t e;
    if ((e = seg(0, first, &g1)) != hipSuccess) return e;
    if ((e = seg(1, body, &g2)) != hipSuccess) return e;
    if ((e = seg(2, tail, &g3)) != hipSuccess) return e;
    if ((e = hipGraphLaunch(g1, d.stream)) != hipSuccess) return e;
    for (int64_t step = 1; step < nsteps; ++step)
      if ((e = hipGraphLaunch(g2, d.stream)) != hipSuccess) return e;
    return hipGraphLaunch(g3, d.stream);
  }

  static hipError_t fft_forward(const DevView& d, void* vpsi) {
    cx<T>* psi = (cx<T>*)vpsi;
    hipError_t e = zpass(d, psi, false, true, 0, 0, 0, 0);
    if (e != hipSuccess) return e;
    if ((e = ypass<false>(d, psi)) != hipSuccess) return e;
    return xpass<XP_FWD>(d, psi, 0, 0);
  }

  // ------------------------------------------------------------ adjoint
  template <bool PI, bool PF>
  static hipError_t za(const DevView& d, const AdjointView& a, int nv, int iv0, int iv1) {
    using SA = typename AdjSched<SC>::type;
    auto k = k3d_zpass_adj<SA, S, CZ, PI, PF>;
    const size_t lds = (size_t)CZ * N * sizeof(cx<double>);
    hipError_t e = set_lds(k, lds);
    if (e != hipSuccess) return e;
    // psi, lambda read + written; per action a table, the eigen table and the
    // gradient accumulator (read + written)
    const double bytes = (4.0 * S + nv * (2.0 * S * (S + 1) / 2.0 + S * (S + 1))) *
                         (double)d.npts * sizeof(cx<double>) / 1.0;
    TimedLaunch tl(d, KIND_OTHER, bytes);
    hipLaunchKernelGGL(k, dim3(N / CZ, N), dim3(CZ * SA::TPC), lds, d.stream,
                       (cx<double>*)a.stacked, (const cx<double>*)d.vexp,
                       (const cx<double>*)a.eig, a.qacc, a.taus, nv, iv0, iv1,
                       (const cx<double>*)d.tw[0]);
    return hipGetLastError();
  }
  static hipError_t zadj(const DevView& d, const AdjointView& a, bool pi, bool pf, int nv,
                         int iv0, int iv1) {
    if (pi && pf) return za<true, true>(d, a, nv, iv0, iv1);
    if (pi) return za<true, false>(d, a, nv, iv0, iv1);
    if (pf) return za<false, true>(d, a, nv, iv0, iv1);
    return za<false, false>(d, a, nv, iv0, iv1);
  }

  // Backward sweep: steps nsteps..1, each step's actions in reverse order
  // with conjugated tables on [psi; lambda]; psi is replaced by the stored
  // checkpoint at every step index that is a multiple of K.
  static hipError_t adjoint_backward(const DevView& d, const AdjointView& a, int64_t nsteps,
                                     int K) {
    if constexpr (!std::is_same<T, double>::value) {
      return hipErrorInvalidValue;
    } else {
      DevView d2 = d;  // the stacked state for the y and x passes
      d2.S = 2 * S;
      cx<T>* stk = (cx<T>*)a.stacked;
      bool zk = false, zopen = false, zpre = false;
      int zv[2] = {0, 0}, znv = 0;
      hipError_t e = hipSuccess;
      auto flush = [&](bool post_fwd) -> hipError_t {
        hipError_t r = zadj(d, a, zpre, post_fwd, znv, zv[0], zv[1]);
        zopen = false;
        znv = 0;
        zk = post_fwd;
        return r;
      };
      for (int64_t n = nsteps; n >= 1; --n) {
        for (int i = d.nact - 1; i >= 0; --i) {
          const int code = d.hprog[i];
          const int idx = prog_idx(code);
          if (prog_op(code) == OP_V) {
            if (zopen && znv == 2) {
              if ((e = flush(false)) != hipSuccess) return e;
            }
            if (!zopen) {
              zopen = true;
              zpre = zk;
              znv = 0;
              zk = false;
            }
            zv[znv++] = idx;
          } else {
            if (zopen) {
              if ((e = flush(true)) != hipSuccess) return e;
            } else if (!zk) {
              if ((e = zadj(d, a, false, true, 0, 0, 0)) != hipSuccess) return e;
              zk = true;
            }
            if ((e = ypass<false>(d2, stk)) != hipSuccess) return e;
            if ((e = xpass<XP_PHASE>(d2, stk, idx, 1)) != hipSuccess) return e;
            if ((e = ypass<true>(d2, stk)) != hipSuccess) return e;
          }
        }
        if ((n - 1) % K == 0) {
          if (zopen) {
            if ((e = flush(false)) != hipSuccess) return e;
          } else if (zk) {
            if ((e = zadj(d, a, true, false, 0, 0, 0)) != hipSuccess) return e;
            zk = false;
          }
          const size_t bytes = (size_t)S * d.npts * sizeof(cx<T>);
          e = hipMemcpyAsync(a.stacked, (const char*)a.checkpoints + (size_t)((n - 1) / K) * bytes,
                             bytes, hipMemcpyDeviceToDevice, d.stream);
          if (e != hipSuccess) return e;
        }
      }
      if (zopen) return flush(false);
      if (zk) return zadj(d, a, true, false, 0, 0, 0);
      return hipSuccess;
    }
  }
};

template <class F>
hipError_t dispatch(int n, int S, bool f64, F&& f) {
#define SOP_3D_CASE(NN)                                                      \
  case NN:                                                                   \
    if (f64) {                                                               \
      if (S == 1) return f.template operator()<double, Z##NN, 1>();          \
      if (S == 2) return f.template operator()<double, Z##NN, 2>();          \
      if (S == 3) return f.template operator()<double, Z##NN, 3>();          \
    } else {                                                                 \
      if (S == 1) return f.template operator()<float, Z##NN, 1>();           \
      if (S == 2) return f.template operator()<float, Z##NN, 2>();           \
      if (S == 3) return f.template operator()<float, Z##NN, 3>();           \
    }                                                                        \
    return hipErrorInvalidValue;
  switch (n) {
    SOP_3D_CASE(32)
    SOP_3D_CASE(48)
    SOP_3D_CASE(64)
    SOP_3D_CASE(128)
    SOP_3D_CASE(256)
    default:
      return hipErrorInvalidValue;
  }
#undef SOP_3D_CASE
}

}  // namespace

int k3d_table_tile(int n, bool f64) {
  (void)n;
  return f64 ? zcols<Z128, double>() : zcols<Z128, float>();
}

bool k3d_plane(int n, bool f64) {
  bool r = false;
  (void)dispatch(n, 1, f64, [&]<typename T, class SC, int S>() -> hipError_t {
    r = Passes<T, SC, S>::PLANE;
    return hipSuccess;
  });
  return r;
}

bool k3d_supported(int n, int S) {
  if (S < 1 || S > 3) return false;
  return n == 32 || n == 48 || n == 64 || n == 128 || n == 256;
}

hipError_t k3d_propagate(const DevView& d, void* psi, int64_t nsteps, int conj) {
  return dispatch(d.n[0], d.S, d.f64, [&]<typename T, class SC, int S>() {
    return Passes<T, SC, S>::propagate(d, psi, nsteps, conj);
  });
}

bool k3d_adjoint_supported(int n, int S, bool f64) {
  return f64 && S >= 1 && S <= 3 && (n == 32 || n == 64 || n == 128 || n == 256);
}

hipError_t k3d_adjoint_backward(const DevView& d, const AdjointView& a, int64_t nsteps, int K) {
  if (!k3d_adjoint_supported(d.n[0], d.S, d.f64)) return hipErrorInvalidValue;
  switch (d.n[0]) {
    case 32:
    case 64:
    case 128:
    case 256:
      break;
    default:
      return hipErrorInvalidValue;
  }
  auto run = [&]<class SC>() -> hipError_t {
    switch (d.S) {
      case 1: return Passes<double, SC, 1>::adjoint_backward(d, a, nsteps, K);
      case 2: return Passes<double, SC, 2>::adjoint_backward(d, a, nsteps, K);
      case 3: return Passes<double, SC, 3>::adjoint_backward(d, a, nsteps, K);
      default: return hipErrorInvalidValue;
    }
  };
  switch (d.n[0]) {
    case 32: return run.template operator()<Z32>();
    case 64: return run.template operator()<Z64>();
    case 128: return run.template operator()<Z128>();
    default: return run.template operator()<Z256>();
  }
}

hipError_t k3d_fft_forward(const DevView& d, void* psi) {
  return dispatch(d.n[0], d.S, d.f64, [&]<typename T, class SC, int S>() {
    return Passes<T, SC, S>::fft_forward(d, psi);
  });
}

}  // namespace sop
