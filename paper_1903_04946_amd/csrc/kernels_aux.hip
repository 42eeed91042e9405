// kernels_aux.hip -- evolution-operator table formation and FP64 reductions.
//
// Potential tables (Sec. "Pruning splitting coefficients": the unique
// evolution operators are computed once at initialisation; Sec. "Molecular
// Hamiltonian in the diabatic basis": the exponential of the S x S potential
// matrix from its Jacobi diagonalisation).  Per grid point the real
// symmetric V(q) is diagonalised by cyclic two-sided Jacobi rotations in
// FP64; for every unique coefficient c the complex-symmetric
// exp(-i tau V/hbar) = R diag(exp(-i lambda tau/hbar)) R^T, tau = c dt, is
// formed in FP64 and rounded once to the plan precision; its packed upper
// triangle is stored structure-of-arrays, [unique][entry][point] for 1D
// grids, or tile-contiguous for the 3D z-pass ([unique][tile][z][entry][col]).
//
// Reductions: norm, surface populations and <V> from psi, <T> from its
// forward transform, and <psi|phi>; every sum is FP64 with a fixed block
// count and a fixed-order tree, so results are bitwise reproducible.
#include "fft_core.hpp"
#include "internal.hpp"

namespace sop {
namespace {

// One sweep set of cyclic Jacobi rotations on a real symmetric S x S matrix.
// On return A is diagonal (eigenvalues on the diagonal) and R holds the
// eigenvectors in its columns.  Each rotation's cosine and sine come from
// the smaller root t = tan(theta) of t^2 + 2 zeta t - 1 = 0, zeta =
// (a_qq - a_pp) / (2 a_pq) (the symmetric Schur step of Golub and Van Loan,
// Matrix Computations, Sec. 8.5): t = sign(zeta) / (|zeta| + sqrt(1 +
// zeta^2)), c = 1 / sqrt(1 + t^2), s = t c -- the rotation with
// tan(2 theta) = 2 a_pq / (a_qq - a_pp), |theta| <= pi/4, without a
// trigonometric call.
template <int S>
__device__ void jacobi_sym(double (&A)[S][S], double (&R)[S][S]) {
#pragma unroll
  for (int i = 0; i < S; ++i)
#pragma unroll
    for (int j = 0; j < S; ++j) R[i][j] = (i == j) ? 1.0 : 0.0;
  if constexpr (S == 1) return;
  for (int sweep = 0; sweep < 24; ++sweep) {
    bool rotated = false;
#pragma unroll
    for (int p = 0; p < S - 1; ++p) {
#pragma unroll
      for (int q = p + 1; q < S; ++q) {
        const double apq = A[p][q];
        if (apq == 0.0) continue;
        const double scale = fabs(A[p][p]) + fabs(A[q][q]);
        if (fabs(apq) <= 1e-18 * scale) {  // negligible next to the diagonal
          A[p][q] = 0.0;
          A[q][p] = 0.0;
          continue;
        }
        rotated = true;
        const double zeta = (A[q][q] - A[p][p]) / (2.0 * apq);
        // 1 / (|zeta| + sqrt(1 + zeta^2)) without overflow for huge zeta
        const double az = fabs(zeta);
        const double tt = az > 1e150 ? 0.5 / az : 1.0 / (az + sqrt(1.0 + az * az));
        const double tn = zeta < 0.0 ? -tt : tt;
        const double cs = 1.0 / sqrt(1.0 + tn * tn);
        const double sn = tn * cs;
        // A <- A J (columns p, q), J = [[c, s], [-s, c]] on (p, q)
#pragma unroll
        for (int r = 0; r < S; ++r) {
          const double arp = A[r][p], arq = A[r][q];
          A[r][p] = cs * arp - sn * arq;
          A[r][q] = sn * arp + cs * arq;
          const double rrp = R[r][p], rrq = R[r][q];
          R[r][p] = cs * rrp - sn * rrq;
          R[r][q] = sn * rrp + cs * rrq;
        }
        // A <- J^T A (rows p, q)
#pragma unroll
        for (int r = 0; r < S; ++r) {
          const double apr = A[p][r], aqr = A[q][r];
          A[p][r] = cs * apr - sn * aqr;
          A[q][r] = sn * apr + cs * aqr;
        }
        A[p][q] = 0.0;
        A[q][p] = 0.0;
      }
    }
    if (!rotated) break;
  }
}

// Destination index of (table u, entry e, point x): structure of arrays for
// 1D (tile = 0) or the z-pass tile layout for a cubic 3D grid of side n.
__device__ __forceinline__ int64_t table_index(int64_t npts, int NE, int tile, int n, int u, int e,
                                               int64_t x) {
  if (tile == 0) return ((int64_t)u * NE + e) * npts + x;
  const int64_t plane = (int64_t)n * n;
  const int64_t z = x / plane, y = (x / n) % n, xx = x % n;
  const int64_t tl = y * (n / tile) + xx / tile;
  return (int64_t)u * NE * npts + tl * ((int64_t)n * NE * tile) + (z * NE + e) * tile + xx % tile;
}

template <typename T, int S>
__global__ void __launch_bounds__(256)
    k_form_vexp(const double* __restrict__ vraw, int64_t npts, const double* __restrict__ taus,
                int ntau, int tile, int n, cx<T>* __restrict__ out,
                const double* __restrict__ dtab, const double* __restrict__ s_dev) {
  constexpr int NE = S * (S + 1) / 2;
  const double sd = dtab ? *s_dev : 0.0;  // driven: V = vraw + s D
  for (int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; x < npts;
       x += (int64_t)gridDim.x * blockDim.x) {
    double A[S][S], R[S][S];
    int e = 0;
#pragma unroll
    for (int i = 0; i < S; ++i)
#pragma unroll
      for (int j = i; j < S; ++j) {
        const int64_t o = (int64_t)e * npts + x;
        const double vij = dtab ? vraw[o] + sd * dtab[o] : vraw[o];
        A[i][j] = vij;
        A[j][i] = vij;
        ++e;
      }
    jacobi_sym<S>(A, R);
    for (int u = 0; u < ntau; ++u) {
      double ere[S], eim[S];
#pragma unroll
      for (int l = 0; l < S; ++l) sincos(-A[l][l] * taus[u], &eim[l], &ere[l]);
      int ee = 0;
#pragma unroll
      for (int i = 0; i < S; ++i)
#pragma unroll
        for (int j = i; j < S; ++j) {
          double re = 0.0, im = 0.0;
#pragma unroll
          for (int l = 0; l < S; ++l) {
            const double rr = R[i][l] * R[j][l];
            re += rr * ere[l];
            im += rr * eim[l];
          }
          const int64_t o = table_index(npts, NE, tile, n, u, ee, x);
          if constexpr (sizeof(T) == 8) {
            out[o] = cx<T>{(T)re, (T)im};
          } else {  // FP32: the pair (rounded, residue) at index 2 o
            const float hr = (float)re, hi = (float)im;
            out[2 * o] = cx<float>{hr, hi};
            out[2 * o + 1] = cx<float>{(float)(re - (double)hr), (float)(im - (double)hi)};
          }
          ++ee;
        }
    }
  }
}

// Block-level fixed-order sum of NV values per thread; thread 0 writes the
// block's NV sums to out.
template <int NV>
__device__ void block_sum(double (&acc)[NV], double* out) {
  __shared__ double red[kReduceThreads][NV];
  const int tid = threadIdx.x;
#pragma unroll
  for (int v = 0; v < NV; ++v) red[tid][v] = acc[v];
  __syncthreads();
  for (int w = kReduceThreads / 2; w > 0; w >>= 1) {
    if (tid < w) {
#pragma unroll
      for (int v = 0; v < NV; ++v) red[tid][v] += red[tid + w][v];
    }
    __syncthreads();
  }
  if (tid == 0) {
#pragma unroll
    for (int v = 0; v < NV; ++v) out[v] = red[0][v];
  }
}

// Per block: sum_x |psi_s(x)|^2 for each s, and sum_x Re(psi(x)^dag V(x) psi(x)).
template <typename T, int S>
__global__ void __launch_bounds__(kReduceThreads)
    k_obs_points(const cx<T>* __restrict__ psi, const double* __restrict__ vraw, int64_t npts,
                 double* __restrict__ partials) {
  double acc[S + 1];
#pragma unroll
  for (int v = 0; v <= S; ++v) acc[v] = 0.0;
  for (int64_t x = (int64_t)blockIdx.x * kReduceThreads + threadIdx.x; x < npts;
       x += (int64_t)gridDim.x * kReduceThreads) {
    double re[S], im[S];
#pragma unroll
    for (int s = 0; s < S; ++s) {
      const cx<T> p = psi[s * npts + x];
      re[s] = (double)p.re;
      im[s] = (double)p.im;
      acc[s] += re[s] * re[s] + im[s] * im[s];
    }
    int e = 0;
    double ev = 0.0;
#pragma unroll
    for (int i = 0; i < S; ++i)
#pragma unroll
      for (int j = i; j < S; ++j) {
        const double vij = vraw[(int64_t)e * npts + x];
        // Re(conj(psi_i) psi_j), counted twice off the diagonal
        const double rr = re[i] * re[j] + im[i] * im[j];
        ev += (i == j ? 1.0 : 2.0) * vij * rr;
        ++e;
      }
    acc[S] += ev;
  }
  block_sum<S + 1>(acc, partials + (size_t)blockIdx.x * (S + 1));
}

// Per block: sum_k T(k) sum_s |psi_hat_s(k)|^2 with T(k) = sum_d inv_mass_d
// (hbar kappa_d)^2 / 2, kappa_d = 2 pi k'_d / (n_d dx_d).
template <typename T>
__global__ void __launch_bounds__(kReduceThreads)
    k_obs_kinetic(const cx<T>* __restrict__ ph, int S, int ndim, int n0, int n1, int n2,
                  double c0, double c1, double c2, double* __restrict__ partials) {
  const int64_t npts = (int64_t)n0 * n1 * n2;
  double acc[1] = {0.0};
  for (int64_t x = (int64_t)blockIdx.x * kReduceThreads + threadIdx.x; x < npts;
       x += (int64_t)gridDim.x * kReduceThreads) {
    const int k2 = (int)(x % n2);
    const int k1 = (int)((x / n2) % n1);
    const int k0 = (int)(x / ((int64_t)n1 * n2));
    auto sq = [](int k, int n) {
      const double kk = (k < n / 2) ? (double)k : (double)(k - n);
      return kk * kk;
    };
    // c_d = inv_mass_d * (hbar * 2 pi / (n_d dx_d))^2 / 2
    double t = c0 * sq(k0, n0);
    if (ndim > 1) t += c1 * sq(k1, n1) + c2 * sq(k2, n2);
    double m = 0.0;
    for (int s = 0; s < S; ++s) {
      const cx<T> p = ph[s * npts + x];
      m += (double)p.re * (double)p.re + (double)p.im * (double)p.im;
    }
    acc[0] += t * m;
  }
  block_sum<1>(acc, partials + blockIdx.x);
}

template <typename T>
__global__ void __launch_bounds__(kReduceThreads)
    k_overlap(const cx<T>* __restrict__ a, const cx<T>* __restrict__ b, int64_t n,
              double* __restrict__ partials) {
  double acc[2] = {0.0, 0.0};
  for (int64_t i = (int64_t)blockIdx.x * kReduceThreads + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * kReduceThreads) {
    const cx<T> p = a[i], q = b[i];
    // conj(p) q
    acc[0] += (double)p.re * (double)q.re + (double)p.im * (double)q.im;
    acc[1] += (double)p.re * (double)q.im - (double)p.im * (double)q.re;
  }
  block_sum<2>(acc, partials + (size_t)blockIdx.x * 2);
}

// sum |a - b|^2 and sum |b|^2, the difference taken in FP64 from the
// stored values.
template <typename T>
__global__ void __launch_bounds__(kReduceThreads)
    k_distance(const cx<T>* __restrict__ a, const cx<T>* __restrict__ b, int64_t n,
               double* __restrict__ partials) {
  double acc[2] = {0.0, 0.0};
  for (int64_t i = (int64_t)blockIdx.x * kReduceThreads + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * kReduceThreads) {
    const cx<T> p = a[i], q = b[i];
    const double dr = (double)p.re - (double)q.re, di = (double)p.im - (double)q.im;
    acc[0] += dr * dr + di * di;
    acc[1] += (double)q.re * (double)q.re + (double)q.im * (double)q.im;
  }
  block_sum<2>(acc, partials + (size_t)blockIdx.x * 2);
}

// Sums nblocks rows of nv partials in a fixed order into out[nv].
__global__ void __launch_bounds__(kReduceThreads)
    k_final(const double* __restrict__ partials, int nblocks, int nv, double* __restrict__ out) {
  __shared__ double red[kReduceThreads];
  for (int v = 0; v < nv; ++v) {
    double acc = 0.0;
    for (int b = threadIdx.x; b < nblocks; b += kReduceThreads) acc += partials[(size_t)b * nv + v];
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int w = kReduceThreads / 2; w > 0; w >>= 1) {
      if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
      __syncthreads();
    }
    if (threadIdx.x == 0) out[v] = red[0];
    __syncthreads();
  }
}

// Compact eigen form of V(q) for the FP64 3D z-pass (S = 2, 3): per point
// the rotation R of V = R diag(lam) R^T (det R = +1, a product of Jacobi
// rotations) and the eigenvalues, in eig_slots(S) complex slots of the
// z-pass tile layout: S = 3 as the unit quaternion (w, x) (y, z) of R and
// (lam_0, lam_1) (lam_2, 0); S = 2 as (cos, sin) of the rotation angle and
// (lam_0, lam_1).  One table serves every coefficient: each potential
// action forms exp(-i tau lam) itself.  The quaternion comes from the
// largest of w^2, x^2, y^2, z^2 (each = (1 +- R_00 +- R_11 +- R_22)/4), so
// the division is always by a number >= 1/2.
template <int S>
__global__ void __launch_bounds__(256)
    k_form_eigq(const double* __restrict__ vraw, int64_t npts, int tile, int n,
                cx<double>* __restrict__ out, const double* __restrict__ dtab,
                const double* __restrict__ s_dev) {
  constexpr int NE = S * (S + 1) / 2;
  constexpr int NQ = eig_slots(S);
  const double sd = dtab ? *s_dev : 0.0;  // driven: V = vraw + s D
  for (int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; x < npts;
       x += (int64_t)gridDim.x * blockDim.x) {
    double A[S][S], R[S][S];
    int e = 0;
#pragma unroll
    for (int i = 0; i < S; ++i)
#pragma unroll
      for (int j = i; j < S; ++j) {
        const int64_t o = (int64_t)e * npts + x;
        const double vij = dtab ? vraw[o] + sd * dtab[o] : vraw[o];
        A[i][j] = vij;
        A[j][i] = vij;
        ++e;
      }
    jacobi_sym<S>(A, R);
    cx<double> slot[NQ];
    if constexpr (S == 2) {
      slot[0] = cx<double>{R[0][0], R[1][0]};
      slot[1] = cx<double>{A[0][0], A[1][1]};
    } else {
      const double t0 = 1.0 + R[0][0] + R[1][1] + R[2][2];  // 4 w^2
      const double t1 = 1.0 + R[0][0] - R[1][1] - R[2][2];  // 4 x^2
      const double t2 = 1.0 - R[0][0] + R[1][1] - R[2][2];  // 4 y^2
      const double t3 = 1.0 - R[0][0] - R[1][1] + R[2][2];  // 4 z^2
      double w, qx, qy, qz;
      if (t0 >= t1 && t0 >= t2 && t0 >= t3) {
        const double r = 2.0 * sqrt(t0);  // 4 w
        w = 0.25 * r;
        qx = (R[2][1] - R[1][2]) / r;
        qy = (R[0][2] - R[2][0]) / r;
        qz = (R[1][0] - R[0][1]) / r;
      } else if (t1 >= t2 && t1 >= t3) {
        const double r = 2.0 * sqrt(t1);  // 4 x
        w = (R[2][1] - R[1][2]) / r;
        qx = 0.25 * r;
        qy = (R[0][1] + R[1][0]) / r;
        qz = (R[0][2] + R[2][0]) / r;
      } else if (t2 >= t3) {
        const double r = 2.0 * sqrt(t2);  // 4 y
        w = (R[0][2] - R[2][0]) / r;
        qx = (R[0][1] + R[1][0]) / r;
        qy = 0.25 * r;
        qz = (R[1][2] + R[2][1]) / r;
      } else {
        const double r = 2.0 * sqrt(t3);  // 4 z
        w = (R[1][0] - R[0][1]) / r;
        qx = (R[0][2] + R[2][0]) / r;
        qy = (R[1][2] + R[2][1]) / r;
        qz = 0.25 * r;
      }
      const double nrm = 1.0 / sqrt(w * w + qx * qx + qy * qy + qz * qz);
      slot[0] = cx<double>{w * nrm, qx * nrm};
      slot[1] = cx<double>{qy * nrm, qz * nrm};
      slot[2] = cx<double>{A[0][0], A[1][1]};
      slot[3] = cx<double>{A[2][2], 0.0};
    }
#pragma unroll
    for (int q = 0; q < NQ; ++q) out[table_index(npts, NQ, tile, n, 0, q, x)] = slot[q];
    (void)NE;
  }
}

// Eigen-decomposition table for the adjoint of one surface: per point the pair
// (R = 1, V) in the z-pass tile layout (two and three surfaces use the compact
// eigen form of k_form_eigq).  Written for any S: R row-major S x S, then the
// eigenvalues, as S(S+1)/2 pairs of doubles.
template <int S>
__global__ void __launch_bounds__(256)
    k_form_eig(const double* __restrict__ vraw, int64_t npts, int tile, int n,
               cx<double>* __restrict__ out) {
  constexpr int NE = S * (S + 1) / 2;
  for (int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; x < npts;
       x += (int64_t)gridDim.x * blockDim.x) {
    double A[S][S], R[S][S];
    int e = 0;
#pragma unroll
    for (int i = 0; i < S; ++i)
#pragma unroll
      for (int j = i; j < S; ++j) {
        const double vij = vraw[(int64_t)e * npts + x];
        A[i][j] = vij;
        A[j][i] = vij;
        ++e;
      }
    jacobi_sym<S>(A, R);
    double flat[2 * NE];
#pragma unroll
    for (int i = 0; i < S; ++i)
#pragma unroll
      for (int j = 0; j < S; ++j) flat[i * S + j] = R[i][j];
#pragma unroll
    for (int l = 0; l < S; ++l) flat[S * S + l] = A[l][l];
#pragma unroll
    for (int q = 0; q < NE; ++q)
      out[table_index(npts, NE, tile, n, 0, q, x)] = cx<double>{flat[2 * q], flat[2 * q + 1]};
  }
}

// vraw = vbase + sum_k delta_k dv_k (the potential is linear in its parameters).
__global__ void __launch_bounds__(256)
    k_vparams(double* __restrict__ vraw, const double* __restrict__ vbase,
              const double* __restrict__ dv, const double* __restrict__ delta, int nparams,
              int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    double v = vbase[i];
    for (int k = 0; k < nparams; ++k) v += delta[k] * dv[(int64_t)k * n + i];
    vraw[i] = v;
  }
}

// lambda_s = w_s psi_s (seed of the adjoint sweep for L = sum_s w_s P_s).
__global__ void __launch_bounds__(256)
    k_scale_surfaces(cx<double>* __restrict__ lam, const cx<double>* __restrict__ psi,
                     const double* __restrict__ w, int S, int64_t npts) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < (int64_t)S * npts;
       i += (int64_t)gridDim.x * blockDim.x) {
    const double ws = w[i / npts];
    lam[i] = cx<double>{ws * psi[i].re, ws * psi[i].im};
  }
}

__global__ void __launch_bounds__(256) k_zero(double* __restrict__ p, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    p[i] = 0.0;
}

// Per block: g_k = sum_x sum_e Q_e(x) dv[k][e][x], k < NP, with Q_e(x) read
// from the accumulator's tile layout [tile (y, x/C)][z][e][x % C] on an n^3
// grid (point x = (z n + y) n + x0).
template <int NP>
__global__ void __launch_bounds__(kReduceThreads)
    k_grad_partials(const double* __restrict__ qacc, const double* __restrict__ dv, int NE,
                    int64_t npts, int n, int cols, double* __restrict__ partials) {
  double acc[NP];
#pragma unroll
  for (int k = 0; k < NP; ++k) acc[k] = 0.0;
  const int64_t plane = (int64_t)n * n;
  for (int64_t x = (int64_t)blockIdx.x * kReduceThreads + threadIdx.x; x < npts;
       x += (int64_t)gridDim.x * kReduceThreads) {
    const int64_t z = x / plane, r = x - z * plane;
    const int64_t y = r / n, x0 = r - y * n;
    const int64_t qb = ((y * (n / cols) + x0 / cols) * n + z) * (int64_t)NE * cols + x0 % cols;
    for (int e = 0; e < NE; ++e) {
      const double q = qacc[qb + (int64_t)e * cols];
#pragma unroll
      for (int k = 0; k < NP; ++k) acc[k] += q * dv[((int64_t)k * NE + e) * npts + x];
    }
  }
  block_sum<NP>(acc, partials + (size_t)blockIdx.x * NP);
}

template <int S, typename T>
hipError_t form_impl(const DevView& d, const double* vraw, const double* taus, int ntau, int tile,
                     void* out, const double* dtab, const double* s_dev) {
  int blocks = (int)((d.npts + 255) / 256);
  if (blocks > 4096) blocks = 4096;
  hipLaunchKernelGGL((k_form_vexp<T, S>), dim3(blocks), dim3(256), 0, d.stream, vraw, d.npts,
                     taus, ntau, tile, d.n[0], (cx<T>*)out, dtab, s_dev);
  return hipGetLastError();
}

template <int S, typename T>
hipError_t obs_points_impl(const DevView& d, const void* psi, const double* vraw,
                           double* partials) {
  hipLaunchKernelGGL((k_obs_points<T, S>), dim3(kReduceBlocks), dim3(kReduceThreads), 0,
                     d.stream, (const cx<T>*)psi, vraw, d.npts, partials);
  return hipGetLastError();
}

}  // namespace

hipError_t form_vexp(const DevView& d, const double* vraw_dev, const double* taus, int ntau,
                     int tile, void* out, const double* dtab, const double* s_dev) {
  switch (d.S) {
    case 1: return d.f64 ? form_impl<1, double>(d, vraw_dev, taus, ntau, tile, out, dtab, s_dev)
                         : form_impl<1, float>(d, vraw_dev, taus, ntau, tile, out, dtab, s_dev);
    case 2: return d.f64 ? form_impl<2, double>(d, vraw_dev, taus, ntau, tile, out, dtab, s_dev)
                         : form_impl<2, float>(d, vraw_dev, taus, ntau, tile, out, dtab, s_dev);
    case 3: return d.f64 ? form_impl<3, double>(d, vraw_dev, taus, ntau, tile, out, dtab, s_dev)
                         : form_impl<3, float>(d, vraw_dev, taus, ntau, tile, out, dtab, s_dev);
    default: return hipErrorInvalidValue;
  }
}

hipError_t form_eigq(const DevView& d, const double* vraw_dev, int tile, void* out,
                     const double* dtab, const double* s_dev) {
  int blocks = (int)((d.npts + 255) / 256);
  if (blocks > 4096) blocks = 4096;
  cx<double>* o = (cx<double>*)out;
  switch (d.S) {
    case 2: hipLaunchKernelGGL(k_form_eigq<2>, dim3(blocks), dim3(256), 0, d.stream, vraw_dev, d.npts, tile, d.n[0], o, dtab, s_dev); break;
    case 3: hipLaunchKernelGGL(k_form_eigq<3>, dim3(blocks), dim3(256), 0, d.stream, vraw_dev, d.npts, tile, d.n[0], o, dtab, s_dev); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

// partials layout: [kReduceBlocks][S+1] for the pointwise sums, then
// [kReduceBlocks] for the kinetic sum.  out_dev receives S + 2 raw sums:
// sum |psi_s|^2 (S values), sum psi^dag V psi, sum T |psi_hat|^2.
hipError_t obs_reduce(const DevView& d, const void* psi, const void* psi_hat,
                      const double* vraw_dev, const double* inv_mass, const double* dx,
                      double hbar, double* partials, double* out_dev) {
  hipError_t e;
  switch (d.S) {
    case 1: e = d.f64 ? obs_points_impl<1, double>(d, psi, vraw_dev, partials)
                      : obs_points_impl<1, float>(d, psi, vraw_dev, partials); break;
    case 2: e = d.f64 ? obs_points_impl<2, double>(d, psi, vraw_dev, partials)
                      : obs_points_impl<2, float>(d, psi, vraw_dev, partials); break;
    case 3: e = d.f64 ? obs_points_impl<3, double>(d, psi, vraw_dev, partials)
                      : obs_points_impl<3, float>(d, psi, vraw_dev, partials); break;
    default: return hipErrorInvalidValue;
  }
  if (e != hipSuccess) return e;
  const int nv = d.S + 1;
  double* kpart = partials + (size_t)kReduceBlocks * nv;
  double c[3] = {0, 0, 0};
  const double twopi = 6.283185307179586476925286766559;
  for (int a = 0; a < d.ndim; ++a) {
    const double kap = hbar * twopi / ((double)d.n[a] * dx[a]);
    c[a] = 0.5 * inv_mass[a] * kap * kap;
  }
  if (d.f64)
    hipLaunchKernelGGL(k_obs_kinetic<double>, dim3(kReduceBlocks), dim3(kReduceThreads), 0,
                       d.stream, (const cx<double>*)psi_hat, d.S, d.ndim, d.n[0], d.n[1], d.n[2],
                       c[0], c[1], c[2], kpart);
  else
    hipLaunchKernelGGL(k_obs_kinetic<float>, dim3(kReduceBlocks), dim3(kReduceThreads), 0,
                       d.stream, (const cx<float>*)psi_hat, d.S, d.ndim, d.n[0], d.n[1], d.n[2],
                       c[0], c[1], c[2], kpart);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  hipLaunchKernelGGL(k_final, dim3(1), dim3(kReduceThreads), 0, d.stream, partials,
                     kReduceBlocks, nv, out_dev);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  hipLaunchKernelGGL(k_final, dim3(1), dim3(kReduceThreads), 0, d.stream, kpart, kReduceBlocks,
                     1, out_dev + nv);
  return hipGetLastError();
}

hipError_t form_eig(const DevView& d, const double* vraw_dev, int tile, void* out) {
  int blocks = (int)((d.npts + 255) / 256);
  if (blocks > 4096) blocks = 4096;
  switch (d.S) {
    case 1: hipLaunchKernelGGL(k_form_eig<1>, dim3(blocks), dim3(256), 0, d.stream, vraw_dev, d.npts, tile, d.n[0], (cx<double>*)out); break;
    // two and three surfaces: the compact eigen form (rotation and eigenvalues)
    case 2:
    case 3: return form_eigq(d, vraw_dev, tile, out, nullptr, nullptr);
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t set_vparams(const DevView& d, double* vraw, const double* vbase, const double* dv,
                       const double* delta_dev, int nparams) {
  const int64_t n = (int64_t)d.S * (d.S + 1) / 2 * d.npts;
  hipLaunchKernelGGL(k_vparams, dim3(2048), dim3(256), 0, d.stream, vraw, vbase, dv, delta_dev,
                     nparams, n);
  return hipGetLastError();
}

hipError_t adjoint_seed(const DevView& d, void* lam, const void* psi, const double* w_dev,
                        double* qacc) {
  hipLaunchKernelGGL(k_scale_surfaces, dim3(2048), dim3(256), 0, d.stream, (cx<double>*)lam,
                     (const cx<double>*)psi, w_dev, d.S, d.npts);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_zero, dim3(2048), dim3(256), 0, d.stream, qacc,
                     (int64_t)d.S * (d.S + 1) / 2 * d.npts);
  return hipGetLastError();
}

hipError_t grad_reduce(const DevView& d, const double* qacc, int cols, const double* dv,
                       int nparams, double* partials, double* out_dev) {
  if (d.ndim != 3 || cols <= 0 || d.n[0] % cols != 0) return hipErrorInvalidValue;
  const int NE = d.S * (d.S + 1) / 2;
  switch (nparams) {
#define SOP_GRAD_CASE(K)                                                                    \
  case K:                                                                                   \
    hipLaunchKernelGGL(k_grad_partials<K>, dim3(kReduceBlocks), dim3(kReduceThreads), 0,    \
                       d.stream, qacc, dv, NE, d.npts, d.n[0], cols, partials);             \
    break;
    SOP_GRAD_CASE(1)
    SOP_GRAD_CASE(2)
    SOP_GRAD_CASE(3)
    SOP_GRAD_CASE(4)
    SOP_GRAD_CASE(5)
    SOP_GRAD_CASE(6)
    SOP_GRAD_CASE(7)
    SOP_GRAD_CASE(8)
#undef SOP_GRAD_CASE
    default:
      return hipErrorInvalidValue;
  }
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_final, dim3(1), dim3(kReduceThreads), 0, d.stream, partials, kReduceBlocks,
                     nparams, out_dev);
  return hipGetLastError();
}

hipError_t pops_reduce(const DevView& d, const void* psi, const double* vraw_dev,
                       double* partials, double* out_dev) {
  hipError_t e;
  switch (d.S) {
    case 1: e = d.f64 ? obs_points_impl<1, double>(d, psi, vraw_dev, partials)
                      : obs_points_impl<1, float>(d, psi, vraw_dev, partials); break;
    case 2: e = d.f64 ? obs_points_impl<2, double>(d, psi, vraw_dev, partials)
                      : obs_points_impl<2, float>(d, psi, vraw_dev, partials); break;
    case 3: e = d.f64 ? obs_points_impl<3, double>(d, psi, vraw_dev, partials)
                      : obs_points_impl<3, float>(d, psi, vraw_dev, partials); break;
    default: return hipErrorInvalidValue;
  }
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_final, dim3(1), dim3(kReduceThreads), 0, d.stream, partials, kReduceBlocks,
                     d.S + 1, out_dev);
  return hipGetLastError();
}

hipError_t distance_reduce(const DevView& d, const void* psi, const void* phi, double* partials,
                           double* out_dev) {
  const int64_t n = d.npts * d.S;
  if (d.f64)
    hipLaunchKernelGGL(k_distance<double>, dim3(kReduceBlocks), dim3(kReduceThreads), 0,
                       d.stream, (const cx<double>*)psi, (const cx<double>*)phi, n, partials);
  else
    hipLaunchKernelGGL(k_distance<float>, dim3(kReduceBlocks), dim3(kReduceThreads), 0,
                       d.stream, (const cx<float>*)psi, (const cx<float>*)phi, n, partials);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_final, dim3(1), dim3(kReduceThreads), 0, d.stream, partials, kReduceBlocks,
                     2, out_dev);
  return hipGetLastError();
}

hipError_t overlap_reduce(const DevView& d, const void* psi, const void* phi, double* partials,
                          double* out_dev) {
  const int64_t n = d.npts * d.S;
  if (d.f64)
    hipLaunchKernelGGL(k_overlap<double>, dim3(kReduceBlocks), dim3(kReduceThreads), 0, d.stream,
                       (const cx<double>*)psi, (const cx<double>*)phi, n, partials);
  else
    hipLaunchKernelGGL(k_overlap<float>, dim3(kReduceBlocks), dim3(kReduceThreads), 0, d.stream,
                       (const cx<float>*)psi, (const cx<float>*)phi, n, partials);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_final, dim3(1), dim3(kReduceThreads), 0, d.stream, partials, kReduceBlocks,
                     2, out_dev);
  return hipGetLastError();
}

}  // namespace sop
