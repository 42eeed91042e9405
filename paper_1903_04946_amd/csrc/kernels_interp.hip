// kernels_interp.hip -- trigonometric interpolation of a grid wavefunction
// onto another uniform grid (Appendix B: wavefunctions on grids of different
// range and density are compared by trigonometric interpolation of the one
// on the sparser grid).
//
// Along one axis the interpolant of samples u_m (m = 0..n-1, x_m = lo + m dx,
// L = n dx) is u(x) = sum_k c_k exp(2 pi i k xi) with xi = (x - lo)/L and
// c_k = (1/n) sum_m u_m exp(-2 pi i k m/n), k over the symmetric band
// |k| < n/2; for even n the Nyquist coefficient enters as c_{n/2} cos(pi n xi),
// so real samples give a real interpolant and the grid points reproduce their
// samples.  Points outside [lo, lo + L) take the value zero (the wavefunction
// is taken to vanish outside the grid it was propagated on).
//
// The interpolant is linear in the samples: along each axis it is a dense
// (n_dst x n_src) complex matrix W, and on a 3D grid the three axis matrices
// act in turn (z, then y, then x).  k_interp_weights forms W on the device in
// FP64; k_cgemm applies it as a batched, strided complex FP64 matrix product
// tiled through LDS (64 x 64 outputs per 256-thread workgroup, 4 x 4 per
// thread, K in slices of 16), the kernel's bound being FP64 arithmetic.
#include "fft_core.hpp"
#include "internal.hpp"

namespace sop {
namespace {

// W[j][m] for destination point j and source sample m.  The position test
// and xi are computed without contraction, in the same order as the plain
// definition (dx_dst = (hi_dst - lo_dst)/n_dst, x = lo_dst + j dx_dst,
// xi = (x - lo)/(hi - lo)), so that a point on the edge is inside or outside
// for every implementation alike.  The phase 2 pi k (xi n - m)/n is reduced
// exactly: xi n = f_i + f_f (integer and fraction), and k (f_i - m) mod n is
// an integer, leaving 2 pi (r + k f_f)/n with |r + k f_f| < 1.5 n.
__global__ void k_interp_weights(double2* __restrict__ W, int n, double lo, double hi, int nd,
                                 double lod, double hid) {
#pragma clang fp contract(off)
  const int m = blockIdx.x * blockDim.x + threadIdx.x;
  const int j = blockIdx.y;
  if (m >= n || j >= nd) return;
  const double dxd = (hid - lod) / nd;
  const double x = lod + j * dxd;
  const double xi = (x - lo) / (hi - lo);
  double2 w = make_double2(0.0, 0.0);
  if (xi >= 0.0 && xi < 1.0) {
    const double f = xi * n;
    const double fi = floor(f);
    const double ff = f - fi;
    const long long d0 = (long long)fi - m;  // integer part of xi n - m
    const int kmax = (n - 1) / 2;            // |k| < n/2
    double re = 0.0, im = 0.0;
    for (int k = -kmax; k <= kmax; ++k) {
      long long r = ((long long)k * d0) % n;
      if (r < 0) r += n;
      const double ph = (2.0 * 3.14159265358979323846) * (((double)r + k * ff) / n);
      double s, c;
      sincos_phase(ph, &s, &c);
      re += c;
      im += s;
    }
    if ((n & 1) == 0) {  // Nyquist: cos(pi (xi n - m)) = (-1)^d0 cos(pi ff)
      double s, c;
      sincos_phase(3.14159265358979323846 * ff, &s, &c);
      re += (d0 & 1) ? -c : c;
    }
    w = make_double2(re / n, im / n);
  }
  W[(size_t)j * n + m] = w;
}

constexpr int BM = 64, BN = 64, BK = 16, NT = 256;

// C[b](i, j) = sum_k A[b](i, k) B[b](k, j), complex FP64, with element strides
// (sai, sak), (sbk, sbj), (sci, scj) and batch strides (bsa, bsb, bsc).
// A_K1: A is contiguous along k (sak = 1), else along i (sai = 1); B_J1: B is
// contiguous along j (sbj = 1), else along k (sbk = 1).  The tile loads put
// the unit-stride index on consecutive lanes.  Out-of-range rows, columns
// and k are loaded as zero and not stored.
template <bool A_K1, bool B_J1>
__global__ __launch_bounds__(NT) void k_cgemm(CgemmArgs g) {
  __shared__ double2 As[BK][BM + 1];
  __shared__ double2 Bs[BK][BN + 1];
  const int t = threadIdx.x;
  const int tx = t % 16, ty = t / 16;
  const int i0 = blockIdx.y * BM, j0 = blockIdx.x * BN;
  const double2* A = g.A + (size_t)blockIdx.z * g.bsa;
  const double2* B = g.B + (size_t)blockIdx.z * g.bsb;
  double2* C = g.C + (size_t)blockIdx.z * g.bsc;
  double2 acc[4][4];
#pragma unroll
  for (int r = 0; r < 4; ++r)
#pragma unroll
    for (int c = 0; c < 4; ++c) acc[r][c] = make_double2(0.0, 0.0);

  for (int k0 = 0; k0 < g.K; k0 += BK) {
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      int i, k;
      if (A_K1) {
        k = t % BK;
        i = t / BK + 16 * q;
      } else {
        i = t % BM;
        k = t / BM + 4 * q;
      }
      const int gi = i0 + i, gk = k0 + k;
      As[k][i] = (gi < g.M && gk < g.K) ? A[(size_t)gi * g.sai + (size_t)gk * g.sak]
                                        : make_double2(0.0, 0.0);
      int jj, kb;
      if (B_J1) {
        jj = t % BN;
        kb = t / BN + 4 * q;
      } else {
        kb = t % BK;
        jj = t / BK + 16 * q;
      }
      const int gj = j0 + jj, gkb = k0 + kb;
      Bs[kb][jj] = (gj < g.N && gkb < g.K) ? B[(size_t)gkb * g.sbk + (size_t)gj * g.sbj]
                                           : make_double2(0.0, 0.0);
    }
    __syncthreads();
#pragma unroll 4
    for (int kk = 0; kk < BK; ++kk) {
      double2 a[4], b[4];
#pragma unroll
      for (int r = 0; r < 4; ++r) a[r] = As[kk][ty + 16 * r];
#pragma unroll
      for (int c = 0; c < 4; ++c) b[c] = Bs[kk][tx + 16 * c];
#pragma unroll
      for (int r = 0; r < 4; ++r)
#pragma unroll
        for (int c = 0; c < 4; ++c) {
          acc[r][c].x = fma(a[r].x, b[c].x, fma(-a[r].y, b[c].y, acc[r][c].x));
          acc[r][c].y = fma(a[r].x, b[c].y, fma(a[r].y, b[c].x, acc[r][c].y));
        }
    }
    __syncthreads();
  }
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const int gi = i0 + ty + 16 * r;
    if (gi >= g.M) continue;
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      const int gj = j0 + tx + 16 * c;
      if (gj < g.N) C[(size_t)gi * g.sci + (size_t)gj * g.scj] = acc[r][c];
    }
  }
}

}  // namespace

hipError_t interp_weights(hipStream_t s, double2* W, int n, double lo, double hi, int nd,
                          double lod, double hid) {
  if (n < 1 || nd < 1 || nd > 65535) return hipErrorInvalidValue;
  dim3 grid((n + 127) / 128, nd);
  hipLaunchKernelGGL(k_interp_weights, grid, dim3(128), 0, s, W, n, lo, hi, nd, lod, hid);
  return hipGetLastError();
}

hipError_t cgemm(hipStream_t s, const CgemmArgs& g, int batch) {
  if (g.M < 1 || g.N < 1 || g.K < 1 || batch < 1 || batch > 65535) return hipErrorInvalidValue;
  const bool a_k1 = g.sak == 1, b_j1 = g.sbj == 1;
  if (!a_k1 && g.sai != 1) return hipErrorInvalidValue;
  if (!b_j1 && g.sbk != 1) return hipErrorInvalidValue;
  const long long gy = (g.M + BM - 1) / BM;
  if (gy > 65535) return hipErrorInvalidValue;
  dim3 grid((g.N + BN - 1) / BN, (unsigned)gy, batch);
  if (a_k1 && b_j1)
    hipLaunchKernelGGL((k_cgemm<true, true>), grid, dim3(NT), 0, s, g);
  else if (a_k1)
    hipLaunchKernelGGL((k_cgemm<true, false>), grid, dim3(NT), 0, s, g);
  else if (b_j1)
    hipLaunchKernelGGL((k_cgemm<false, true>), grid, dim3(NT), 0, s, g);
  else
    hipLaunchKernelGGL((k_cgemm<false, false>), grid, dim3(NT), 0, s, g);
  return hipGetLastError();
}

}  // namespace sop
