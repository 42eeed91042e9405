// passes_3d.hpp -- pencil schedules and the bodies of the pass kinds of the
// 3D executor, as device functions of one workgroup tile.  The kernels of a
// single plan (kernels_3d.hip) and of a batch of plans (kernels_batch3d.hip)
// wrap the same bodies, so both compute identical values.
//
// The kinetic propagator of a separable T(p) = sum_d p_d^2 / (2 m_d) factors
// over the axes: exp(-i tau T / hbar) = K_z K_y K_x with the commuting
// one-dimensional actions K_d = F_d^-1 diag(f_d) F_d along axis d (Sec.
// "Dynamic Fourier method": the kinetic action is diagonal in the momentum
// representation, and both it and the FFT factor over the axes).  A substep
// (one potential action followed by one kinetic action) is therefore three
// passes over psi[s][z][y][x], each taking the state from and back to the
// position representation:
//   z-pass : potential unitary(ies) -> forward FFT z -> f_z -> inverse FFT z
//            (all S surfaces of a tile of x-columns: the S x S matvec of
//            Sec. "Molecular Hamiltonian in the diabatic basis" runs in
//            registers);
//   y-pass : forward FFT y -> f_y -> inverse FFT y;
//   x-pass : forward FFT x -> f_x -> inverse FFT x.
// Where the whole xy plane fits in LDS the y- and x-passes run as one plane
// pass.  The per-axis factor f_d(k) = exp(-i tau hbar kappa_k^2 / (2 m_d)) / n_d
// carries the 1/n_d of the unnormalised inverse transform.
#pragma once

#include "fft_core.hpp"
#include "internal.hpp"

namespace sop {
namespace s3d {

using Z32 = Sched<32, 8, RList<8, 4>, RList<4, 8>, 8, 4>;
using Z48 = Sched<48, 12, RList<4, 4, 3>, RList<3, 4, 4>, 4, 3>;
using Z64 = Sched<64, 8, RList<8, 8>, RList<8, 8>, 8, 8>;
using Z128 = Sched<128, 8, RList<8, 4, 4>, RList<4, 4, 8>, 8, 4>;
using Z256 = Sched<256, 8, RList<8, 8, 4>, RList<4, 8, 8>, 8, 4>;

// Schedules of the single-pencil y and x passes: sixteen values per thread
// where that saves an LDS exchange.
template <class SC>
struct XYSched {
  using type = SC;
};
template <>
struct XYSched<Z128> {
  using type = Sched<128, 16, RList<16, 8>, RList<8, 16>, 16, 8>;
};
template <>
struct XYSched<Z256> {
  using type = Sched<256, 16, RList<16, 16>, RList<16, 16>, 16, 16>;
};

// Columns per tile of the y-pass: at least a full wave per block and
// 128-byte contiguous row segments.
template <class SC, typename T>
constexpr int cols() {
  constexpr int seg = 128 / (int)sizeof(cx<T>);
  return SC::TPC * seg >= 64 ? seg : 64 / SC::TPC;
}

// Rows per x-pass block: about 128 threads, and a divisor of N.
template <class XS>
constexpr int xrows() {
  int r = XS::TPC >= 16 ? 8 : 128 / XS::TPC;
  while (XS::N % r != 0) r /= 2;
  return r;
}

// Column width of the potential-table tiles (and of the default z-pass tile):
// 16 in both precisions, 256-byte FP64 and 128-byte FP32 segments of psi.
constexpr int kTableCols = 16;

}  // namespace s3d

// Complex entries of one axis block of the twiddle and factor tables (in FP32
// the (rounded, residue) pairs of Split<float>).
template <typename T, int N>
constexpr int axis_block() {
  return N * Split<T>::rep;
}

// LDS of the y-pass tiles (C columns) and of the x-pass tiles (ROWS rows):
// the exchange area and two staged axis blocks (twiddles, factor).  The
// z-pass reads its twiddles and factor from global memory: with the
// potential's table reads in flight, staging them measured slower (57.2
// against 54.8 us a pass for 128^3 x 3 FP64), while it saves 4-5% on the
// y-, x- and plane passes.
template <typename T, int N>
constexpr size_t y_lds_elems(int C) {
  return (size_t)C * N + 2 * axis_block<T, N>();
}
template <typename T, int N>
constexpr size_t x_lds_elems(int ROWS) {
  return (size_t)ROWS * (N + N / 16) + 2 * axis_block<T, N>();
}

// Copies nb axis blocks (src[b], axis_block entries each) into LDS at dst,
// every thread of the block striding over them.  The y-, x- and plane passes
// stage their twiddles and kinetic factors this way before loading their
// pencils: every later read of them is an LDS read instead of a dependent
// global load in the middle of the transform.  Every transform starts with a
// stage that uses no twiddles, followed by an LDS exchange whose barrier
// orders these writes before the first read.
// `lane` and `nt` are the thread's index in the tile and the tile's thread
// count.
template <typename T, int N, int NB>
__device__ __forceinline__ void stage_blocks(cx<T>* dst, const cx<T>* const (&src)[NB], int lane,
                                             int nt) {
  constexpr int A = axis_block<T, N>();
  for (int i = lane; i < A; i += nt) {
#pragma unroll
    for (int b = 0; b < NB; ++b) dst[b * A + i] = src[b][i];
  }
}

// What a pass does along its axis after its pointwise work:
//   AX_NONE: nothing (z-pass carrying only potential actions);
//   AX_KIN : forward FFT -> per-axis kinetic factor -> inverse FFT;
//   AX_FWD : forward FFT only, output in the momentum representation (the
//            observables' transform).
enum { AX_NONE = 0, AX_KIN = 1, AX_FWD = 2 };

// v (forward-transformed, radix-RL ownership) *= f[k] (conjugated factor
// when conj): the kinetic factor of one axis (a split block in FP32).
template <typename T, class SC, int P>
__device__ __forceinline__ void axis_phase(cx<T> (*v)[SC::E], const cx<T>* __restrict__ f,
                                           T csign, int t) {
#pragma unroll
  for (int q = 0; q < SC::E; ++q) {
    const Fac<T> w = load_fac(f, own_idx<SC::N, SC::E, SC::RL>(t, q), csign);
#pragma unroll
    for (int p = 0; p < P; ++p) v[p][q] = fmul(v[p][q], w);
  }
}

// ---------------------------------------------------------------- z-pass
// Potential tables are stored per tile of TC x-columns: for table u, tile
// (y, x / TC) holds [z][entry][x % TC] contiguously, N * NE * TC complex, so
// a tile reads its table as one contiguous stream.  The pass tile is C
// columns wide (C divides TC); block (bx, by) owns columns bx*C .. bx*C+C-1
// of row y = by.  `psi` is one state [S][N^3]; `fz` the z factor of the
// kinetic set (AX_KIN only).
//
// Table entries are cx<T>, in FP32 the pairs (rounded, residue) of
// Split<float> (each entry's index doubled).  `lane` (here and in the y- and
// x-pass bodies) is the thread's index in the tile, threadIdx.x unless a
// persistent caller passes it through opaque() so that the compiler does not
// keep every lane-derived offset live across its work loop.  `src` (here and
// there): where the pass reads the state, psi itself when NULL (in place);
// the pass always writes psi.
//
// EQ (S = 2, 3): `vexp` is instead the one compact eigen-form table, FP64 in
// both precisions (eig_slots(S) complex double slots per point, same tile
// layout), and `taus` the tau of each coefficient; a potential action is
// psi <- R exp(-i tau lam) R^T psi in registers, and the two actions at a
// step boundary share one load, one pair of rotations and one phase
// (psi <- R exp(-i (tau_1 + tau_2) lam) R^T psi: the same operator, rounded
// once).  The action is computed in FP64 in both precisions: an FP32 state
// is widened, rotated and phased in FP64 and rounded once, so the FP32 form
// carries no rounded potential operator.
// cache-policy bits of a buffer load: non-temporal
constexpr int kCpolNT = 2;

template <typename T, int S>
__device__ __forceinline__ void rotation_from_slots(const cx<T>* q, T (&R)[S][S]) {
  if constexpr (S == 2) {
    const T c = q[0].re, s = q[0].im;
    R[0][0] = c;
    R[0][1] = -s;
    R[1][0] = s;
    R[1][1] = c;
  } else {
    const T w = q[0].re, x = q[0].im, y = q[1].re, z = q[1].im;
    R[0][0] = (T)1 - (T)2 * (y * y + z * z);
    R[0][1] = (T)2 * (x * y - z * w);
    R[0][2] = (T)2 * (x * z + y * w);
    R[1][0] = (T)2 * (x * y + z * w);
    R[1][1] = (T)1 - (T)2 * (x * x + z * z);
    R[1][2] = (T)2 * (y * z - x * w);
    R[2][0] = (T)2 * (x * z - y * w);
    R[2][1] = (T)2 * (y * z + x * w);
    R[2][2] = (T)1 - (T)2 * (x * x + y * y);
  }
}

template <typename T, class SC, int S, int C, int TC, int AX, bool EQ = false>
__device__ __forceinline__ void zpass_body(cx<T>* __restrict__ psi,
                                           const void* __restrict__ vexp, int nv, int iv0,
                                           int iv1, int conj, const cx<T>* __restrict__ tw,
                                           const cx<T>* __restrict__ fz, cx<T>* lds, int bx,
                                           int by, const double* __restrict__ taus = nullptr,
                                           int lane = (int)threadIdx.x,
                                           const cx<T>* src = nullptr) {
  static_assert(TC % C == 0, "pass tile must divide the table tile");
  static_assert(!EQ || S >= 2, "eigen form: two or three surfaces");
  constexpr int N = SC::N, E = SC::E, NE = EQ ? eig_slots(S) : S * (S + 1) / 2;
  const int col = lane % C, t = lane / C;
  const int x = bx * C + col, y = by;
  constexpr uint32_t plane = (uint32_t)N * N;
  constexpr int64_t npts = (int64_t)plane * N;
  constexpr uint32_t tile = (uint32_t)N * NE * TC;
  const uint32_t off0 = (uint32_t)y * N + x;
  const int tx = (C == TC) ? bx : (bx * C) / TC;            // table tile
  const int tcol = (C == TC) ? col : (bx * C) % TC + col;   // column within it
  const size_t tbase = ((size_t)y * (N / TC) + tx) * tile;
  const LayStrided lay{col, 0, C};  // one surface at a time through LDS
  cx<T> v[S][E];
  const cx<T>* const in = src ? src : psi;
#pragma unroll
  for (int s = 0; s < S; ++s) {
    const auto rs = rsrc(in + s * npts, (uint32_t)npts);
#pragma unroll
    for (int q = 0; q < E; ++q) v[s][q] = ld<T>(rs, own_idx<N, E, SC::RF>(t, q) * plane + off0);
  }
  const T csign = conj ? (T)-1 : (T)1;
  if constexpr (EQ) {
    if (nv >= 1) {
      const auto rq = rsrc((const cx<double>*)vexp + tbase, tile);
      // two actions at a step boundary: exp(-i tau_2 lam) exp(-i tau_1 lam)
      // = exp(-i (tau_1 + tau_2) lam), one phase per eigenvalue
      const double tab = (double)csign * (taus[iv0] + (nv >= 2 ? taus[iv1] : 0.0));
#pragma unroll
      for (int q = 0; q < E; ++q) {
        const uint32_t pt = (uint32_t)own_idx<N, E, SC::RF>(t, q) * (NE * TC) + tcol;
        cx<double> sl[NE];
#pragma unroll
        for (int e = 0; e < NE; ++e) {
          // an eigen table larger than the last-level cache (256^3: 1.07 GB)
          // is read with the non-temporal hint: read once a pass, it would
          // only evict the state from the caches
          const sop_u32x4 w = __builtin_amdgcn_raw_buffer_load_b128(
              rq, (int)((pt + e * TC) * 16u), 0, N >= 256 ? kCpolNT : 0);
          sl[e] = __builtin_bit_cast(cx<double>, w);
        }
        double R[S][S];
        rotation_from_slots<double, S>(sl, R);
        const double lam[3] = {sl[S == 3 ? 2 : 1].re, sl[S == 3 ? 2 : 1].im,
                               S == 3 ? sl[NE - 1].re : 0.0};
        // gamma = R^T psi, gamma_k *= exp(-i tau lam_k) per action, psi = R gamma
        cx<double> g[S];
#pragma unroll
        for (int k = 0; k < S; ++k) {
          g[k] = cx<double>{0.0, 0.0};
#pragma unroll
          for (int i = 0; i < S; ++i)
            g[k] = cx<double>{g[k].re + R[i][k] * (double)v[i][q].re,
                              g[k].im + R[i][k] * (double)v[i][q].im};
          double sn, cs;
          sincos_phase(tab * lam[k], &sn, &cs);
          g[k] = cmul(g[k], cx<double>{cs, -sn});
        }
#pragma unroll
        for (int i = 0; i < S; ++i) {
          cx<double> a = {0.0, 0.0};
#pragma unroll
          for (int k = 0; k < S; ++k)
            a = cx<double>{a.re + R[i][k] * g[k].re, a.im + R[i][k] * g[k].im};
          v[i][q] = cx<T>{(T)a.re, (T)a.im};
        }
      }
    }
  } else {
    constexpr int REP = Split<T>::rep;
    auto vact = [&](int iv) {
      const auto ru = rsrc((const cx<T>*)vexp + ((size_t)iv * NE * npts + tbase) * REP,
                           tile * REP);
#pragma unroll
      for (int q = 0; q < E; ++q) {
        const uint32_t pt = (uint32_t)own_idx<N, E, SC::RF>(t, q) * (NE * TC) + tcol;
        Fac<T> u[NE];
#pragma unroll
        for (int e = 0; e < NE; ++e) u[e] = ldfac<T>(ru, pt + e * TC, csign);
        cx<T> w[S];
#pragma unroll
        for (int s = 0; s < S; ++s) w[s] = v[s][q];
        apply_u_fac<T, S>(w, u);
#pragma unroll
        for (int s = 0; s < S; ++s) v[s][q] = w[s];
      }
    };
    if (nv >= 1) vact(iv0);
    if (nv >= 2) vact(iv1);
  }
  if constexpr (AX != AX_NONE) {
#pragma unroll
    for (int s = 0; s < S; ++s) fft_forward<SC, 1>(v + s, lds, lay, tw, t);
  }
  if constexpr (AX == AX_KIN) {
    axis_phase<T, SC, S>(v, fz, csign, t);
#pragma unroll
    for (int s = 0; s < S; ++s) fft_inverse<SC, 1>(v + s, lds, lay, tw, t);
  }
  constexpr int ROUT = AX == AX_FWD ? SC::RL : SC::RF;
#pragma unroll
  for (int s = 0; s < S; ++s) {
    const auto rs = rsrc(psi + s * npts, (uint32_t)npts);
#pragma unroll
    for (int q = 0; q < E; ++q) st(rs, own_idx<N, E, ROUT>(t, q) * plane + off0, v[s][q]);
  }
}

// ---------------------------------------------------------------- y-pass
// One surface `psi_s` [N^3]; block (bx, z) owns columns bx*C .. bx*C+C-1 of
// plane z.  AX = AX_KIN (factor fy) or AX_FWD.
template <typename T, class SC, int C, int AX>
__device__ __forceinline__ void ypass_body(cx<T>* __restrict__ psi_s,
                                           const cx<T>* __restrict__ tw,
                                           const cx<T>* __restrict__ fy, int conj, cx<T>* lds,
                                           int bx, int z, int lane = (int)threadIdx.x,
                                           const cx<T>* src_s = nullptr) {
  constexpr int N = SC::N, E = SC::E;
  const int col = lane % C, t = lane / C;
  const int x = bx * C + col;
  constexpr int64_t plane = (int64_t)N * N;
  const auto base = rsrc(psi_s + z * plane, (uint32_t)plane);
  const auto bin = rsrc((src_s ? src_s : psi_s) + z * plane, (uint32_t)plane);
  const LayStrided lay{col, 0, C};
  cx<T>* const tws = lds + C * N;  // staged twiddles and y factor
  if constexpr (AX == AX_KIN) {
    stage_blocks<T, N, 2>(tws, {tw, fy}, lane, C * SC::TPC);
  } else {
    stage_blocks<T, N, 1>(tws, {tw}, lane, C * SC::TPC);
  }
  cx<T> v[1][E];
#pragma unroll
  for (int q = 0; q < E; ++q) v[0][q] = ld<T>(bin, own_idx<N, E, SC::RF>(t, q) * N + x);
  fft_forward<SC, 1>(v, lds, lay, tws, t);
  if constexpr (AX == AX_KIN) {
    axis_phase<T, SC, 1>(v, tws + axis_block<T, N>(), conj ? (T)-1 : (T)1, t);
    fft_inverse<SC, 1>(v, lds, lay, tws, t);
  }
  constexpr int ROUT = AX == AX_FWD ? SC::RL : SC::RF;
#pragma unroll
  for (int q = 0; q < E; ++q) st(base, own_idx<N, E, ROUT>(t, q) * N + x, v[0][q]);
}

// ---------------------------------------------------------------- x-pass
// One surface `psi_s`; block (bx, z) owns rows bx*ROWS .. bx*ROWS+ROWS-1 of
// plane z.  AX = AX_KIN (factor fx) or AX_FWD.
template <typename T, class SC, int ROWS, int AX>
__device__ __forceinline__ void xpass_body(cx<T>* __restrict__ psi_s,
                                           const cx<T>* __restrict__ tw,
                                           const cx<T>* __restrict__ fx, int conj, cx<T>* lds,
                                           int bx, int z, int lane = (int)threadIdx.x,
                                           const cx<T>* src_s = nullptr) {
  constexpr int N = SC::N, E = SC::E, TPC = SC::TPC;
  const int t = lane % TPC, row = lane / TPC;
  const int y = bx * ROWS + row;
  constexpr int64_t plane = (int64_t)N * N;
  const auto base = rsrc(psi_s + z * plane, (uint32_t)plane);
  const auto bin = rsrc((src_s ? src_s : psi_s) + z * plane, (uint32_t)plane);
  const uint32_t yo = (uint32_t)y * N;
  const LayPadded lay{row * (N + N / 16), 0};
  cx<T>* const tws = lds + ROWS * (N + N / 16);  // staged twiddles and x factor
  if constexpr (AX == AX_KIN) {
    stage_blocks<T, N, 2>(tws, {tw, fx}, lane, ROWS * TPC);
  } else {
    stage_blocks<T, N, 1>(tws, {tw}, lane, ROWS * TPC);
  }
  cx<T> v[1][E];
#pragma unroll
  for (int q = 0; q < E; ++q) v[0][q] = ld<T>(bin, own_idx<N, E, SC::RF>(t, q) + yo);
  fft_forward<SC, 1>(v, lds, lay, tws, t);
  if constexpr (AX == AX_KIN) {
    axis_phase<T, SC, 1>(v, tws + axis_block<T, N>(), conj ? (T)-1 : (T)1, t);
    fft_inverse<SC, 1>(v, lds, lay, tws, t);
  }
  constexpr int ROUT = AX == AX_FWD ? SC::RL : SC::RF;
#pragma unroll
  for (int q = 0; q < E; ++q) st(base, own_idx<N, E, ROUT>(t, q) + yo, v[0][q]);
}

// ---------------------------------------------------------------- xy plane
// The y- and x-passes of one kinetic action fused for grids whose whole xy
// plane fits in LDS: block = one plane z of one surface, N x TPC threads.
// The y round trip runs in the column layout (lane -> x = lane % N,
// t = lane / N), one LDS transpose moves the plane to the row layout
// (lane -> t = lane % TPC, y = lane / TPC), where the x round trip runs and
// the rows are stored.  Every pencil sees the same stages, twiddles and
// factors as in the separate passes, so the values are identical.
template <typename T, class SC>
constexpr size_t plane_lds_elems() {
  return (size_t)SC::N * (SC::N + SC::N / 16) + 4 * axis_block<T, SC::N>();
}
template <typename T, class SC>
constexpr bool plane_fits() {
  return plane_lds_elems<T, SC>() * sizeof(cx<T>) <= 160 * 1024 && SC::N * SC::TPC <= 1024;
}

// `kin` = the three per-axis factors [f_z | f_y | f_x] of one kinetic set.
template <typename T, class SC>
__device__ __forceinline__ void plane_body(cx<T>* __restrict__ psi_s,
                                           const cx<T>* __restrict__ tw,
                                           const cx<T>* __restrict__ kin, int conj, cx<T>* lds,
                                           int z) {
  constexpr int N = SC::N, E = SC::E, TPC = SC::TPC;
  constexpr int P = N + N / 16;  // padded row stride in LDS
  const int lane = threadIdx.x;
  const int col = lane % N, tc = lane / N;    // column layout
  const int tr = lane % TPC, row = lane / TPC;  // row layout
  constexpr int64_t plane = (int64_t)N * N;
  const auto base = rsrc(psi_s + z * plane, (uint32_t)plane);
  constexpr int AS = axis_block<T, N>();  // axis stride of the twiddle and factor blocks
  // staged [twiddles y | twiddles x | f_y | f_x] after the plane
  cx<T>* const twy = lds + N * P;
  cx<T>* const twx = twy + AS;
  stage_blocks<T, N, 4>(twy, {tw + AS, tw + 2 * AS, kin + AS, kin + 2 * AS}, lane, N * TPC);
  const LayStrided lcol{col, 0, N};
  const LayPadded lrow{row * P, 0};
  const T csign = conj ? (T)-1 : (T)1;
  cx<T> v[1][E];
  // y round trip (columns)
#pragma unroll
  for (int q = 0; q < E; ++q) v[0][q] = ld<T>(base, own_idx<N, E, SC::RF>(tc, q) * N + col);
  fft_forward<SC, 1>(v, lds, lcol, twy, tc);
  axis_phase<T, SC, 1>(v, twy + 2 * AS, csign, tc);
  fft_inverse<SC, 1>(v, lds, lcol, twy, tc);
  // columns -> rows
#pragma unroll
  for (int q = 0; q < E; ++q) lds[own_idx<N, E, SC::RF>(tc, q) * P + col] = v[0][q];
  __syncthreads();
#pragma unroll
  for (int q = 0; q < E; ++q) v[0][q] = lds[row * P + own_idx<N, E, SC::RF>(tr, q)];
  __syncthreads();
  // x round trip (rows)
  fft_forward<SC, 1>(v, lds, lrow, twx, tr);
  axis_phase<T, SC, 1>(v, twy + 3 * AS, csign, tr);
  fft_inverse<SC, 1>(v, lds, lrow, twx, tr);
#pragma unroll
  for (int q = 0; q < E; ++q) st(base, row * N + own_idx<N, E, SC::RF>(tr, q), v[0][q]);
}

}  // namespace sop
