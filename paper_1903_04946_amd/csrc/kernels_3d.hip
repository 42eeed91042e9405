// kernels_3d.hip -- three-dimensional cubic grids n^3: the composed time step
// as a sequence of pencil passes over psi[s][z][y][x] (x fastest).
//
// A substep (one potential action followed by one kinetic action, Sec.
// "Dynamic Fourier method") is three passes over the state, each from and
// back to the position representation (the kinetic propagator factors over
// the axes, see passes_3d.hpp):
//   z-pass : potential unitary(ies) -> forward FFT z -> f_z -> inverse FFT z
//            (all S surfaces of a tile of x-columns, so the S x S matvec of
//            Sec. "Molecular Hamiltonian in the diabatic basis" runs in
//            registers);
//   y-pass : forward FFT y -> f_y -> inverse FFT y;
//   x-pass : forward FFT x -> f_x -> inverse FFT x;
// or, where the xy plane fits in LDS, the z-pass and one plane pass.  The
// last potential action of a step and the first of the next share one
// z-pass (two matvecs in registers; the arithmetic is the same as two
// separate passes).  The planner stores the three per-axis factors
// f_d = exp(-i tau hbar kappa^2 / (2 m_d)) / n_d of each unique coefficient.
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

// Columns per tile of the z-pass: the table tile width, or half of it
//   on 64^3, where 16-column tiles give one workgroup per compute unit
//   (smaller grids keep 16 columns: half a tile would be half a wave);
//   on 256^3, where 16 columns make 512-thread workgroups of ~200 VGPRs
//   (two per SIMD); 256-thread ones schedule better (556 vs 586 us a pass
//   for 256^3 x 3 FP64).
template <class SC, typename T>
constexpr int zcols() {
  if (SC::N == 64 && SC::TPC * kTableCols / 2 >= 64) return kTableCols / 2;
  if (SC::N == 256) return kTableCols / 2;
  return kTableCols;
}

// ---------------------------------------------------------------- z-pass
// grid (N / C, N, states); fz = the z factor of the kinetic set (AX_KIN)
// EQ: the potential comes from the compact eigen form (FP64 table, S >= 2).
template <typename T, class SC, int S, int C, int AX, bool EQ>
__global__ void __launch_bounds__(C * SC::TPC)
    k3d_zpass(cx<T>* __restrict__ psi, const void* __restrict__ vexp, int nv, int iv0, int iv1,
              int conj, const cx<T>* __restrict__ tw, const cx<T>* __restrict__ fz,
              const double* __restrict__ taus, const cx<T>* src) {
  extern __shared__ char smem_raw[];
  cx<T>* lds = reinterpret_cast<cx<T>*>(smem_raw);
  const size_t off = (size_t)blockIdx.z * S * ((size_t)SC::N * SC::N * SC::N);  // member
  zpass_body<T, SC, S, C, kTableCols, AX, EQ>(psi + off, vexp, nv, iv0, iv1, conj, tw, fz, lds,
                                              blockIdx.x, blockIdx.y, taus, (int)threadIdx.x,
                                              src ? src + off : nullptr);
}

// ---------------------------------------------------------------- adjoint z-pass
// Backward sweep of the adjoint method over the stacked state [psi; lambda]
// (2S pencils, FP64).  For each potential action j, walked in reverse, the
// kernel holds psi_j (the state after the action) and lambda_j (the adjoint
// after it) and, with V(x) = R diag(lam) R^T read from the eigen table (for
// two and three surfaces the compact form: R as a unit quaternion or a
// rotation angle's (cos, sin), and the eigenvalues; for one surface (1, V)) and
// D = diag(exp(-i tau lam)), computes in eigen coordinates
//   psi_{j-1} = U_j^dag psi_j = R conj(D) R^T psi_j,
//   lambda_{j-1} = U_j^dag lambda_j = R conj(D) R^T lambda_j,
//   Q(x) += R Re(M) R^T,  M_ab = conj(alpha_a) F_ab beta_b,
// with alpha = R^T lambda_j, beta = R^T psi_{j-1} and the divided
// differences of f(v) = exp(-i tau v):
//   F_ab = (f(lam_a) - f(lam_b)) / (lam_a - lam_b)
//        = -i tau exp(-i tau (lam_a + lam_b)/2) sinc(tau (lam_a - lam_b)/2),
// so that d P / d theta_k = 2 dV sum_x sum_ij Q_ij(x) D_k,ij(x) (Daleckii-
// Krein form of the Frechet derivative of exp(-i tau V(theta))).  Q is kept
// packed (Q_ii; Q_ij + Q_ji for i < j) and tile-contiguous like the tables,
// qacc[tile (y, x/C)][z][entry][x % C], so that a workgroup's accumulator
// reads and writes are whole contiguous runs (C * S(S+1)/2 doubles per z)
// rather than C-double segments of S(S+1)/2 separate arrays.  With KZ the
// pass then applies the adjoint z factor K_z^dag (conjugated f_z) to all 2S
// pencils.
// The pass tile is C columns of the TC-column table tiles (C divides TC).
// Two waves per SIMD: with six pencils of state the three-surface pass needs
// about 200-250 VGPRs, and a one-wave budget let the compiler take more.
template <class SC, int S, int C, int TC, bool KZ>
__global__ void __launch_bounds__(C * SC::TPC) __attribute__((amdgpu_waves_per_eu(2)))
    k3d_zpass_adj(cx<double>* __restrict__ stk, const cx<double>* __restrict__ eig,
                  double* __restrict__ qacc,
                  const double* __restrict__ taus, int nv, int iv0, int iv1,
                  const cx<double>* __restrict__ tw, const cx<double>* __restrict__ fz) {
  static_assert(TC % C == 0, "pass tile must divide the table tile");
  extern __shared__ char smem_raw[];
  cx<double>* lds = reinterpret_cast<cx<double>*>(smem_raw);
  constexpr int N = SC::N, E = SC::E, NE = S * (S + 1) / 2, P = 2 * S;
  constexpr int NQ = S >= 2 ? eig_slots(S) : 1;  // eigen-table slots per point
  const int lane = threadIdx.x;
  const int col = lane % C, t = lane / C;
  const int x = blockIdx.x * C + col, y = blockIdx.y;
  constexpr uint32_t plane = (uint32_t)N * N;
  constexpr int64_t npts = (int64_t)plane * N;
  constexpr uint32_t tile = (uint32_t)N * NQ * TC;
  const uint32_t off0 = (uint32_t)y * N + x;
  const int tcol = (blockIdx.x * C) % TC + col;  // column within the table tile
  const size_t tbase = ((size_t)y * (N / TC) + (blockIdx.x * C) / TC) * tile;
  const LayStrided lay{col, 0, C};
  double* const qbase = qacc + ((size_t)y * (N / C) + blockIdx.x) * ((size_t)N * NE * C) + col;
  cx<double> v[P][E];
#pragma unroll
  for (int s = 0; s < P; ++s) {
    const auto rs = rsrc(stk + s * npts, (uint32_t)npts);
#pragma unroll
    for (int q = 0; q < E; ++q)
      v[s][q] = ld<double>(rs, own_idx<N, E, SC::RF>(t, q) * plane + off0);
  }
  auto vact = [&](int iv) {
    const auto rg = rsrc(eig + tbase, tile);
    const double tau = taus[iv];
#pragma unroll
    for (int q = 0; q < E; ++q) {
      const uint32_t tp = (uint32_t)own_idx<N, E, SC::RF>(t, q) * (NQ * TC) + tcol;
      double ev[S * S + S];  // R (row-major S x S) then lam (S)
      {
        cx<double> sl[NQ];
#pragma unroll
        for (int e = 0; e < NQ; ++e) sl[e] = ld<double>(rg, tp + e * TC);
        if constexpr (S == 1) {
          ev[0] = 1.0;
          ev[1] = sl[0].im;
        } else {
          double R[S][S];
          rotation_from_slots<double, S>(sl, R);
#pragma unroll
          for (int i = 0; i < S; ++i)
#pragma unroll
            for (int j = 0; j < S; ++j) ev[i * S + j] = R[i][j];
          ev[S * S] = sl[S == 3 ? 2 : 1].re;
          ev[S * S + 1] = sl[S == 3 ? 2 : 1].im;
          if constexpr (S == 3) ev[S * S + 2] = sl[NQ - 1].re;
        }
      }
      // eigen coordinates: gamma = R^T psi_j, alpha = R^T lambda_j
      cx<double> ga[S], al[S];
#pragma unroll
      for (int a = 0; a < S; ++a) {
        ga[a] = cx<double>{0.0, 0.0};
        al[a] = cx<double>{0.0, 0.0};
#pragma unroll
        for (int i = 0; i < S; ++i) {
          const double r = ev[i * S + a];
          ga[a] = cx<double>{ga[a].re + r * v[i][q].re, ga[a].im + r * v[i][q].im};
          al[a] = cx<double>{al[a].re + r * v[S + i][q].re, al[a].im + r * v[S + i][q].im};
        }
      }
      const double* lam = ev + S * S;
      // c_a = exp(-i tau lam_a / 2): three sincos per point instead of one per
      // (a, b) pair.  exp(-i tau (lam_a + lam_b)/2) = c_a c_b and
      // exp(i h_ab) = c_b conj(c_a) with h_ab = tau (lam_a - lam_b)/2, so
      // sin(h_ab) = Im(c_b conj(c_a)); below |h| = 1e-2 the sinc comes from its
      // series (the product form would lose relative accuracy there).
      cx<double> c[S];
#pragma unroll
      for (int a = 0; a < S; ++a) {
        double sn, cs;
        sincos_phase(0.5 * tau * lam[a], &sn, &cs);
        c[a] = cx<double>{cs, -sn};
      }
      // U_j^dag = R conj(D) R^T with D_a = exp(-i tau lam_a) = c_a^2:
      // beta = R^T psi_{j-1} = conj(D) gamma, formed in place of gamma (the
      // temporaries of one point are kept few: with the six pencils of the
      // stacked state they decide how many waves a SIMD holds)
#pragma unroll
      for (int a = 0; a < S; ++a) ga[a] = cmul(cconj(cmul(c[a], c[a])), ga[a]);
      // T = R Re(M) with M_ab = conj(alpha_a) F_ab beta_b, accumulated entry by
      // entry (F_ab = -i tau exp(-i tau (lam_a + lam_b)/2) sinc(tau (lam_a - lam_b)/2))
      // sinc(h_ab) is symmetric in (a, b): one value per pair a < b, chosen
      // without a branch between the series and the quotient
      double sinc[S][S];
#pragma unroll
      for (int a = 0; a < S; ++a) {
        sinc[a][a] = 1.0;
#pragma unroll
        for (int b = a + 1; b < S; ++b) {
          const double h = 0.5 * tau * (lam[a] - lam[b]);
          const double h2 = h * h;
          const double ser = 1.0 - h2 * (1.0 / 6.0 - h2 * (1.0 / 120.0 - h2 * (1.0 / 5040.0)));
          const double sh = c[b].im * c[a].re - c[b].re * c[a].im;  // Im(c_b conj(c_a))
          const double quo = sh / h;
          sinc[a][b] = sinc[b][a] = fabs(h) < 1e-2 ? ser : quo;
        }
      }
      double tq[S][S];
#pragma unroll
      for (int i = 0; i < S; ++i)
#pragma unroll
        for (int b = 0; b < S; ++b) tq[i][b] = 0.0;
#pragma unroll
      for (int a = 0; a < S; ++a)
#pragma unroll
        for (int b = 0; b < S; ++b) {
          const double sc = sinc[a][b];
          const cx<double> e2 = cmul(c[a], c[b]);
          // -i tau sc e2
          const cx<double> F = {tau * sc * e2.im, -tau * sc * e2.re};
          const cx<double> fb = cmul(F, ga[b]);
          const double rm = al[a].re * fb.re + al[a].im * fb.im;  // Re(M_ab)
#pragma unroll
          for (int i = 0; i < S; ++i) tq[i][b] += ev[i * S + a] * rm;
        }
      // Q = T R^T, accumulated packed.  The point's accumulator address is
      // made to depend on T, so that its loads are not issued ahead of the
      // point's arithmetic (held across it, they cost the pass its registers)
      uint32_t qo = (uint32_t)own_idx<N, E, SC::RF>(t, q) * (NE * C);
      asm volatile("" : "+v"(qo) : "v"(tq[0][0]));
      double* const qp0 = qbase + qo;
      int e = 0;
#pragma unroll
      for (int i = 0; i < S; ++i)
#pragma unroll
        for (int j = i; j < S; ++j) {
          double qij = 0.0, qji = 0.0;
#pragma unroll
          for (int b = 0; b < S; ++b) {
            qij += tq[i][b] * ev[j * S + b];
            qji += tq[j][b] * ev[i * S + b];
          }
          qp0[e * C] += (i == j) ? qij : qij + qji;
          ++e;
        }
      // psi_{j-1} = R beta, lambda_{j-1} = R conj(D) alpha
#pragma unroll
      for (int a = 0; a < S; ++a) al[a] = cmul(cconj(cmul(c[a], c[a])), al[a]);
#pragma unroll
      for (int i = 0; i < S; ++i) {
        cx<double> p = {0.0, 0.0}, l = {0.0, 0.0};
#pragma unroll
        for (int a = 0; a < S; ++a) {
          const double r = ev[i * S + a];
          p = cx<double>{p.re + r * ga[a].re, p.im + r * ga[a].im};
          l = cx<double>{l.re + r * al[a].re, l.im + r * al[a].im};
        }
        v[i][q] = p;
        v[S + i][q] = l;
      }
    }
  };
  if (nv >= 1) vact(iv0);
  if (nv >= 2) vact(iv1);
  if constexpr (KZ) {
#pragma unroll
    for (int s = 0; s < P; ++s) fft_forward<SC, 1>(v + s, lds, lay, tw, t);
    axis_phase<double, SC, P>(v, fz, -1.0, t);
#pragma unroll
    for (int s = 0; s < P; ++s) fft_inverse<SC, 1>(v + s, lds, lay, tw, t);
  }
#pragma unroll
  for (int s = 0; s < P; ++s) {
    const auto rs = rsrc(stk + s * npts, (uint32_t)npts);
#pragma unroll
    for (int q = 0; q < E; ++q) st(rs, own_idx<N, E, SC::RF>(t, q) * plane + off0, v[s][q]);
  }
}

// ---------------------------------------------------------------- y-pass
// grid (N / C, N, surfaces x states): blockIdx.z picks one surface pencil set;
// fy = the y factor of the kinetic set (AX_KIN)
template <typename T, class SC, int C, int AX>
__global__ void __launch_bounds__(C * SC::TPC)
    k3d_ypass(cx<T>* __restrict__ psi, const cx<T>* __restrict__ tw,
              const cx<T>* __restrict__ fy, int conj, const cx<T>* src) {
  extern __shared__ char smem_raw[];
  cx<T>* lds = reinterpret_cast<cx<T>*>(smem_raw);
  constexpr int64_t npts = (int64_t)SC::N * SC::N * SC::N;
  ypass_body<T, SC, C, AX>(psi + blockIdx.z * npts, tw, fy, conj, lds, blockIdx.x, blockIdx.y,
                           (int)threadIdx.x, src ? src + blockIdx.z * npts : nullptr);
}

// ---------------------------------------------------------------- x-pass
// grid (N / ROWS, N, surfaces x states); fx = the x factor (AX_KIN)
template <typename T, class SC, int ROWS, int AX>
__global__ void __launch_bounds__(ROWS * SC::TPC)
    k3d_xpass(cx<T>* __restrict__ psi, const cx<T>* __restrict__ tw,
              const cx<T>* __restrict__ fx, int conj, const cx<T>* src) {
  extern __shared__ char smem_raw[];
  cx<T>* lds = reinterpret_cast<cx<T>*>(smem_raw);
  constexpr int64_t npts = (int64_t)SC::N * SC::N * SC::N;
  xpass_body<T, SC, ROWS, AX>(psi + blockIdx.z * npts, tw, fx, conj, lds, blockIdx.x, blockIdx.y,
                              (int)threadIdx.x, src ? src + blockIdx.z * npts : nullptr);
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
// Pass program of the 3D executor.  The machine walks the step program
// (forward, or reversed for the adjoint sweep): potential actions are held
// (up to two) until a kinetic action closes them into one z-pass that also
// carries that action's z factor, followed by its y- and x-passes (or its
// plane pass); potential actions still held at the end of the run form a
// z-pass of their own.
struct PassMachine {
  int zv[2] = {0, 0}, znv = 0;
  bool operator==(const PassMachine& o) const {
    return znv == o.znv && (znv < 1 || zv[0] == o.zv[0]) && (znv < 2 || zv[1] == o.zv[1]);
  }
};

void flush_z(PassMachine& m, bool kz, int tidx, std::vector<PassDesc>& out) {
  PassDesc p;
  p.kind = PassDesc::Z;
  p.kz = kz;
  p.tidx = tidx;
  p.nv = m.znv;
  p.iv0 = m.zv[0];
  p.iv1 = m.zv[1];
  out.push_back(p);
  m.znv = 0;
}

// One action of the program: code = prog_entry(op, table index).
void emit_action(PassMachine& m, int code, std::vector<PassDesc>& out, bool xy) {
  const int idx = prog_idx(code);
  if (prog_op(code) == OP_V) {
    if (m.znv == 2) flush_z(m, false, 0, out);
    m.zv[m.znv++] = idx;
    return;
  }
  flush_z(m, true, idx, out);
  PassDesc p;
  p.tidx = idx;
  if (xy) {
    p.kind = PassDesc::XY;
    out.push_back(p);
    return;
  }
  p.kind = PassDesc::Y;
  out.push_back(p);
  p.kind = PassDesc::X;
  out.push_back(p);
}

void emit_step(const DevView& d, PassMachine& m, std::vector<PassDesc>& out, bool xy) {
  for (int a = 0; a < d.nact; ++a) emit_action(m, d.hprog[a], out, xy);
}

void emit_flush(PassMachine& m, std::vector<PassDesc>& out) {
  if (m.znv > 0) flush_z(m, false, 0, out);
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

  // the potential may come from the compact eigen form (one table for every
  // coefficient; plans whose phases stay within kPhaseMax)
  static constexpr bool EQ = eig_form(3, S);

  // algorithmic bytes of one pass: psi read + written (d.S pencil sets: the
  // adjoint's y- and x-passes run on the stacked 2S), plus tables read (the
  // FP64 eigen form is read once for up to two actions; FP32 table entries
  // are (rounded, residue) pairs)
  static double pass_bytes(const DevView& d, int ntables) {
    const double tab = (EQ && d.eig) ? (ntables > 0 ? eig_slots(S) * sizeof(cx<double>) : 0.0)
                                     : ntables * S * (S + 1) / 2.0 * sizeof(cx<T>) *
                                           Split<T>::rep;
    return (2.0 * d.S * sizeof(cx<T>) + tab) * (double)d.npts * d.count;
  }
  // axis factor a (0 z, 1 y, 2 x) of kinetic set tidx
  static const cx<T>* kfac(const DevView& d, int tidx, int a) {
    return (const cx<T>*)d.kin + ((size_t)tidx * 3 + a) * d.kin_stride;
  }

  template <int AX>
  static hipError_t z(const DevView& d, cx<T>* psi, int nv, int iv0, int iv1, int tidx,
                      int conj, const cx<T>* src = nullptr) {
    if constexpr (EQ) {
      if (d.eig) return zk<AX, true>(d, psi, nv, iv0, iv1, tidx, conj, src);
    }
    return zk<AX, false>(d, psi, nv, iv0, iv1, tidx, conj, src);
  }
  template <int AX, bool Q>
  static hipError_t zk(const DevView& d, cx<T>* psi, int nv, int iv0, int iv1, int tidx,
                       int conj, const cx<T>* src) {
    auto k = k3d_zpass<T, SC, S, CZ, AX, Q>;
    const size_t lds = (size_t)CZ * N * sizeof(cx<T>);
    hipError_t e = set_lds(k, lds);
    if (e != hipSuccess) return e;
    TimedLaunch tl(d, KIND_ZPASS, pass_bytes(d, nv));
    hipLaunchKernelGGL(k, dim3(N / CZ, N, d.count), dim3(CZ * SC::TPC), lds, d.stream, psi,
                       d.vexp, nv, iv0, iv1, conj, (const cx<T>*)d.tw[0],
                       AX == AX_KIN ? kfac(d, tidx, 0) : nullptr, d.vtaus, src);
    return hipGetLastError();
  }
  template <int AX>
  static hipError_t ypass(const DevView& d, cx<T>* psi, int tidx, int conj,
                          const cx<T>* src = nullptr) {
    auto k = k3d_ypass<T, XS, C, AX>;
    const size_t lds = y_lds_elems<T, N>(C) * sizeof(cx<T>);
    hipError_t e = set_lds(k, lds);
    if (e != hipSuccess) return e;
    TimedLaunch tl(d, KIND_YPASS, pass_bytes(d, 0));
    hipLaunchKernelGGL(k, dim3(N / C, N, d.S * d.count), dim3(C * XS::TPC), lds, d.stream, psi,
                       (const cx<T>*)d.tw[1], AX == AX_KIN ? kfac(d, tidx, 1) : nullptr, conj,
                       src);
    return hipGetLastError();
  }
  template <int AX>
  static hipError_t xpass(const DevView& d, cx<T>* psi, int tidx, int conj,
                          const cx<T>* src = nullptr) {
    auto k = k3d_xpass<T, XS, ROWS, AX>;
    const size_t lds = x_lds_elems<T, N>(ROWS) * sizeof(cx<T>);
    hipError_t e = set_lds(k, lds);
    if (e != hipSuccess) return e;
    TimedLaunch tl(d, KIND_XPASS, pass_bytes(d, 0));
    hipLaunchKernelGGL(k, dim3(N / ROWS, N, d.S * d.count), dim3(ROWS * XS::TPC), lds,
                       d.stream, psi, (const cx<T>*)d.tw[2],
                       AX == AX_KIN ? kfac(d, tidx, 2) : nullptr, conj, src);
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
      TimedLaunch tl(d, KIND_PLANE, pass_bytes(d, 0));
      hipLaunchKernelGGL(k, dim3(N, d.S * d.count), dim3(N * XS::TPC), lds, d.stream, psi,
                         (const cx<T>*)d.tw[0], kfac(d, tidx, 0), conj);
      return hipGetLastError();
    }
  }

  // Launches one pass descriptor.
  static hipError_t launch(const DevView& d, cx<T>* psi, const PassDesc& p, int conj) {
    switch (p.kind) {
      case PassDesc::Z:
        return p.kz ? z<AX_KIN>(d, psi, p.nv, p.iv0, p.iv1, p.tidx, conj)
                    : z<AX_NONE>(d, psi, p.nv, p.iv0, p.iv1, 0, conj);
      case PassDesc::Y: return ypass<AX_KIN>(d, psi, p.tidx, conj);
      case PassDesc::X: return xpass<AX_KIN>(d, psi, p.tidx, conj);
      default: return plane(d, psi, p.tidx, conj);
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
    hipGraphExec_t g1, g2, g3 = nullptr;
    hipError_t e;
    if ((e = seg(0, first, &g1)) != hipSuccess) return e;
    if ((e = seg(1, body, &g2)) != hipSuccess) return e;
    if (!tail.empty() && (e = seg(2, tail, &g3)) != hipSuccess) return e;
    if ((e = hipGraphLaunch(g1, d.stream)) != hipSuccess) return e;
    for (int64_t step = 1; step < nsteps; ++step)
      if ((e = hipGraphLaunch(g2, d.stream)) != hipSuccess) return e;
    return g3 ? hipGraphLaunch(g3, d.stream) : hipSuccess;
  }

  // Forward transform of every surface (momentum representation, natural
  // order, unnormalised) for the observables.
  static hipError_t fft_forward(const DevView& d, void* vpsi) {
    cx<T>* psi = (cx<T>*)vpsi;
    hipError_t e = z<AX_FWD>(d, psi, 0, 0, 0, 0, 0);
    if (e != hipSuccess) return e;
    if ((e = ypass<AX_FWD>(d, psi, 0, 0)) != hipSuccess) return e;
    return xpass<AX_FWD>(d, psi, 0, 0);
  }

  // ------------------------------------------------------------ adjoint
  // Columns per adjoint z-pass tile: 256 threads per block, but at least 8
  // columns (128-byte row segments; 512 threads at 256^3, two waves per SIMD
  // as the register budget allows).  The gradient accumulator's tiles have
  // this width.
  static constexpr int kAdjCA0 = (256 / AdjSched<SC>::type::TPC < kTableCols)
                                     ? 256 / AdjSched<SC>::type::TPC
                                     : kTableCols;
  static constexpr int kAdjCols = kAdjCA0 < 8 ? 8 : kAdjCA0;

  template <bool KZ>
  static hipError_t za(const DevView& d, const AdjointView& a, int nv, int iv0, int iv1,
                       int tidx) {
    using SA = typename AdjSched<SC>::type;
    constexpr int CA = kAdjCols;
    auto k = k3d_zpass_adj<SA, S, CA, kTableCols, KZ>;
    const size_t lds = (size_t)CA * N * sizeof(cx<double>);
    hipError_t e = set_lds(k, lds);
    if (e != hipSuccess) return e;
    // psi, lambda read + written; per action the eigen table (eig_slots(S)
    // complex for S >= 2, one for S = 1) and the gradient accumulator
    // (S(S+1)/2 doubles, read + written)
    constexpr double NE = S * (S + 1) / 2.0;
    constexpr double NQ = S >= 2 ? eig_slots(S) : 1;
    const double bytes = ((4.0 * S + nv * NQ) * sizeof(cx<double>) +
                          nv * 2.0 * NE * sizeof(double)) * (double)d.npts;
    TimedLaunch tl(d, KIND_OTHER, bytes);
    hipLaunchKernelGGL(k, dim3(N / CA, N), dim3(CA * SA::TPC), lds, d.stream,
                       (cx<double>*)a.stacked, (const cx<double>*)a.eig, a.qacc, a.taus, nv,
                       iv0, iv1,
                       (const cx<double>*)d.tw[0],
                       KZ ? (const cx<double>*)kfac(d, tidx, 0) : nullptr);
    return hipGetLastError();
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
      PassMachine m;
      std::vector<PassDesc> ps;
      auto run = [&]() -> hipError_t {
        for (const PassDesc& p : ps) {
          hipError_t r;
          switch (p.kind) {
            case PassDesc::Z:
              r = p.kz ? za<true>(d, a, p.nv, p.iv0, p.iv1, p.tidx)
                       : za<false>(d, a, p.nv, p.iv0, p.iv1, 0);
              break;
            case PassDesc::Y: r = ypass<AX_KIN>(d2, stk, p.tidx, 1); break;
            default: r = xpass<AX_KIN>(d2, stk, p.tidx, 1); break;
          }
          if (r != hipSuccess) return r;
        }
        ps.clear();
        return hipSuccess;
      };
      hipError_t e = hipSuccess;
      for (int64_t n = nsteps; n >= 1; --n) {
        for (int i = d.nact - 1; i >= 0; --i) emit_action(m, d.hprog[i], ps, false);
        if ((n - 1) % K == 0) {
          emit_flush(m, ps);
          if ((e = run()) != hipSuccess) return e;
          const size_t bytes = (size_t)S * d.npts * sizeof(cx<T>);
          e = hipMemcpyAsync(a.stacked, (const char*)a.checkpoints + (size_t)((n - 1) / K) * bytes,
                             bytes, hipMemcpyDeviceToDevice, d.stream);
          if (e != hipSuccess) return e;
          if (d.timer) d.timer->break_chain();
        } else if ((e = run()) != hipSuccess) {
          return e;
        }
      }
      emit_flush(m, ps);
      return run();
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
  (void)f64;
  return kTableCols;
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
  if (d.timer) d.timer->break_chain();  // untimed work may precede this call
  return dispatch(d.n[0], d.S, d.f64, [&]<typename T, class SC, int S>() {
    return Passes<T, SC, S>::propagate(d, psi, nsteps, conj);
  });
}

hipError_t k3d_axis_kinetic(const DevView& d, void* psi, int axis, const void* src) {
  if (d.timer) d.timer->break_chain();
  return dispatch(d.n[0], d.S, d.f64, [&]<typename T, class SC, int S>() -> hipError_t {
    using P = Passes<T, SC, S>;
    cx<T>* v = (cx<T>*)psi;
    const cx<T>* u = (const cx<T>*)src;
    switch (axis) {
      case 0: return P::template z<AX_KIN>(d, v, 0, 0, 0, 0, 0, u);
      case 1: return P::template ypass<AX_KIN>(d, v, 0, 0, u);
      case 2: return P::template xpass<AX_KIN>(d, v, 0, 0, u);
      default: return hipErrorInvalidValue;
    }
  });
}

bool k3d_adjoint_supported(int n, int S, bool f64) {
  return f64 && S >= 1 && S <= 3 && (n == 32 || n == 64 || n == 128 || n == 256);
}

int k3d_adjoint_cols(int n) {
  switch (n) {
    case 32: return Passes<double, Z32, 1>::kAdjCols;
    case 64: return Passes<double, Z64, 1>::kAdjCols;
    case 128: return Passes<double, Z128, 1>::kAdjCols;
    case 256: return Passes<double, Z256, 1>::kAdjCols;
    default: return 0;
  }
}

hipError_t k3d_adjoint_backward(const DevView& d, const AdjointView& a, int64_t nsteps, int K) {
  if (d.timer) d.timer->break_chain();  // untimed work may precede this call
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
  if (d.timer) d.timer->break_chain();  // untimed work may precede this call
  return dispatch(d.n[0], d.S, d.f64, [&]<typename T, class SC, int S>() {
    return Passes<T, SC, S>::fft_forward(d, psi);
  });
}

}  // namespace sop
