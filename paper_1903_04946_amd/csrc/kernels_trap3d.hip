// kernels_trap3d.hip -- pointwise and reduction kernels of the trapezoidal
// rule on 3D grids (FP64).
//
// A stage of the trapezoidal rule solves (1 + i tau H) x = (1 - i tau H) psi
// with the conjugate orthogonal conjugate gradient method (H is real
// symmetric on the grid, so 1 + i tau H is complex symmetric).  On a 3D grid
// the kinetic part of H p is the sum of three one-axis terms,
// T p = sum_d F_d^-1 T_d(k) F_d p, each computed by the pass kernels of the
// propagator on its own copy of p with the factor T_d(k)/n_d in place of the
// phase (the host sequences them); the kernels here add the three terms and
// the S x S matvec with V(x), form A p = p + i tau H p, update the iterates,
// and reduce the inner products the method needs (u^T v without conjugation,
// and |u|^2) in a fixed order: block partials, then one final block.
//
// The iteration's scalars live on the device (the status block `st`, see
// T3 below): the final blocks form rho, mu, |r|^2 and the convergence test,
// and the update kernels read alpha = rho / mu and beta = rho_new / rho from
// it, so the host only reads the status every few iterations.  Once the
// residual test holds (or mu breaks down) the status freezes the iterate:
// later iterations of the block use alpha = beta = 0 and leave x unchanged.
#include "fft_core.hpp"
#include "internal.hpp"

namespace sop {
namespace {

typedef cx<double> cd_t;

constexpr int kTB = kReduceThreads;  // threads per block
constexpr int kNB = kReduceBlocks;   // blocks (grid-stride over the points)

__device__ __forceinline__ cd_t cmuli(cd_t a, double t) { return {-t * a.im, t * a.re}; }  // i t a

// Fixed-order block sum of NV values; thread 0 writes them to out.
template <int NV>
__device__ void tsum(double (&acc)[NV], double* out) {
  __shared__ double red[kTB][NV];
  const int tid = threadIdx.x;
#pragma unroll
  for (int v = 0; v < NV; ++v) red[tid][v] = acc[v];
  __syncthreads();
  for (int w = kTB / 2; w > 0; w >>= 1) {
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

// h_s = qz_s + qy_s + qx_s + sum_r V_sr u_r at point x (all surfaces).
template <int S>
__device__ __forceinline__ void hvec(const cd_t* __restrict__ qz, const cd_t* __restrict__ qy,
                                     const cd_t* __restrict__ qx, const cd_t* __restrict__ u,
                                     const double* __restrict__ vraw, int64_t npts, int64_t x,
                                     cd_t (&in)[S], cd_t (&h)[S]) {
#pragma unroll
  for (int s = 0; s < S; ++s) in[s] = u[s * npts + x];
#pragma unroll
  for (int s = 0; s < S; ++s) {
    const int64_t o = s * npts + x;
    cd_t a = cadd(cadd(qz[o], qy[o]), qx[o]);
#pragma unroll
    for (int r = 0; r < S; ++r) {
      const int i = s < r ? s : r, j = s < r ? r : s;
      const double v = vraw[(int64_t)(i * S - i * (i - 1) / 2 + (j - i)) * npts + x];
      a = {fma(v, in[r].re, a.re), fma(v, in[r].im, a.im)};
    }
    h[s] = a;
  }
}

// Start of a stage from x = psi: h = H x, b = x - i tau h, r = b - A x =
// -2 i tau h, p = r.  Partials: |b|^2, |r|^2, r^T r (re, im).
template <int S>
__global__ void __launch_bounds__(kTB)
    k_t3_init(const cd_t* __restrict__ qz, const cd_t* __restrict__ qy,
              const cd_t* __restrict__ qx, const cd_t* __restrict__ x,
              const double* __restrict__ vraw, int64_t npts, double tau, cd_t* __restrict__ r,
              cd_t* __restrict__ p, double* __restrict__ partials) {
  double acc[4] = {0.0, 0.0, 0.0, 0.0};
  for (int64_t i = (int64_t)blockIdx.x * kTB + threadIdx.x; i < npts;
       i += (int64_t)gridDim.x * kTB) {
    cd_t in[S], h[S];
    hvec<S>(qz, qy, qx, x, vraw, npts, i, in, h);
#pragma unroll
    for (int s = 0; s < S; ++s) {
      const cd_t b = csub(in[s], cmuli(h[s], tau));
      const cd_t rr = cmuli(h[s], -2.0 * tau);
      r[s * npts + i] = rr;
      p[s * npts + i] = rr;
      acc[0] += b.re * b.re + b.im * b.im;
      acc[1] += rr.re * rr.re + rr.im * rr.im;
      acc[2] += rr.re * rr.re - rr.im * rr.im;
      acc[3] += 2.0 * rr.re * rr.im;
    }
  }
  tsum<4>(acc, partials + (size_t)blockIdx.x * 4);
}

// ap = A p = p + i tau H p.  Partials: p^T ap (re, im).
template <int S>
__global__ void __launch_bounds__(kTB)
    k_t3_ap(const cd_t* __restrict__ qz, const cd_t* __restrict__ qy,
            const cd_t* __restrict__ qx, const cd_t* __restrict__ p,
            const double* __restrict__ vraw, int64_t npts, double tau, cd_t* __restrict__ ap,
            double* __restrict__ partials) {
  double acc[2] = {0.0, 0.0};
  for (int64_t i = (int64_t)blockIdx.x * kTB + threadIdx.x; i < npts;
       i += (int64_t)gridDim.x * kTB) {
    cd_t in[S], h[S];
    hvec<S>(qz, qy, qx, p, vraw, npts, i, in, h);
#pragma unroll
    for (int s = 0; s < S; ++s) {
      const cd_t a = cadd(in[s], cmuli(h[s], tau));
      ap[s * npts + i] = a;
      acc[0] += in[s].re * a.re - in[s].im * a.im;
      acc[1] += in[s].re * a.im + in[s].im * a.re;
    }
  }
  tsum<2>(acc, partials + (size_t)blockIdx.x * 2);
}

// x += alpha p, r -= alpha ap with alpha = rho / mu from the status (0 once
// it is frozen).  Partials: |r|^2, r^T r (re, im).
__device__ __forceinline__ cd_t cdiv(double are, double aim, double bre, double bim) {
  const double den = bre * bre + bim * bim;
  return {(are * bre + aim * bim) / den, (aim * bre - are * bim) / den};
}

__global__ void __launch_bounds__(kTB)
    k_t3_update(cd_t* __restrict__ x, cd_t* __restrict__ r, const cd_t* __restrict__ p,
                const cd_t* __restrict__ ap, int64_t n, const double* __restrict__ st,
                double* __restrict__ partials) {
  const cd_t alpha = st[T3_STOP] != 0.0 ? cd_t{0.0, 0.0}
                                        : cdiv(st[T3_RHO], st[T3_RHO + 1], st[T3_MU],
                                               st[T3_MU + 1]);
  double acc[3] = {0.0, 0.0, 0.0};
  for (int64_t i = (int64_t)blockIdx.x * kTB + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * kTB) {
    x[i] = cadd(x[i], cmul(alpha, p[i]));
    const cd_t rn = csub(r[i], cmul(alpha, ap[i]));
    r[i] = rn;
    acc[0] += rn.re * rn.re + rn.im * rn.im;
    acc[1] += rn.re * rn.re - rn.im * rn.im;
    acc[2] += 2.0 * rn.re * rn.im;
  }
  tsum<3>(acc, partials + (size_t)blockIdx.x * 3);
}

// p = r + beta p with beta = rho_new / rho from the status (0 once frozen).
__global__ void __launch_bounds__(kTB)
    k_t3_pupdate(const cd_t* __restrict__ r, cd_t* __restrict__ p, int64_t n,
                 const double* __restrict__ st) {
  const cd_t beta = st[T3_STOP] != 0.0 ? cd_t{0.0, 0.0}
                                       : cdiv(st[T3_RHO_NEW], st[T3_RHO_NEW + 1], st[T3_RHO],
                                              st[T3_RHO + 1]);
  for (int64_t i = (int64_t)blockIdx.x * kTB + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * kTB)
    p[i] = cadd(r[i], cmul(beta, p[i]));
}

// out[v] = sum over the kNB blocks of partials[b][v], in a fixed order (in
// thread 0), then thread 0 applies `post` to the status with the sums.
template <int NV, class Post>
__device__ void final_sum(const double* __restrict__ partials, Post post) {
  __shared__ double red[kTB];
  double out[NV];
  for (int v = 0; v < NV; ++v) {
    double acc = 0.0;
    for (int b = threadIdx.x; b < kNB; b += kTB) acc += partials[(size_t)b * NV + v];
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int w = kTB / 2; w > 0; w >>= 1) {
      if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
      __syncthreads();
    }
    out[v] = red[0];
    __syncthreads();
  }
  if (threadIdx.x == 0) post(out);
}

// Start of a stage: |b|^2, |r|^2 and rho = r^T r; converged at once if
// |r|^2 <= tol^2 |b|^2.
__global__ void __launch_bounds__(kTB)
    k_t3_final_init(const double* __restrict__ partials, double tol2, int max_iter,
                    double* __restrict__ st) {
  final_sum<4>(partials, [&](const double* o) {
    st[T3_MAXIT] = (double)max_iter;
    st[T3_BB] = o[0];
    st[T3_RR] = o[1];
    st[T3_RHO] = st[T3_RHO_NEW] = o[2];
    st[T3_RHO + 1] = st[T3_RHO_NEW + 1] = o[3];
    st[T3_TOL2] = tol2;
    st[T3_STOP] = o[1] <= tol2 * o[0] ? 1.0 : 0.0;
    st[T3_ITER] = 0.0;
    st[T3_FAIL] = 0.0;
  });
}

// mu = p^T A p for this iteration, after rho takes the value of the last
// update; a zero or non-finite mu is a breakdown (stop, failed).
__global__ void __launch_bounds__(kTB)
    k_t3_final_ap(const double* __restrict__ partials, double* __restrict__ st) {
  final_sum<2>(partials, [&](const double* o) {
    if (st[T3_STOP] != 0.0) return;
    st[T3_RHO] = st[T3_RHO_NEW];
    st[T3_RHO + 1] = st[T3_RHO_NEW + 1];
    const double mabs = fabs(o[0]) + fabs(o[1]);
    if (!(mabs > 0.0) || !(mabs < 1e300)) {
      st[T3_FAIL] = 1.0;
      st[T3_STOP] = 1.0;
      return;
    }
    st[T3_MU] = o[0];
    st[T3_MU + 1] = o[1];
  });
}

// After the update: one more iteration, |r|^2, rho_new, the test, and the
// iteration limit (stop there; the host sees |r|^2 above the bar).
__global__ void __launch_bounds__(kTB)
    k_t3_final_update(const double* __restrict__ partials, double* __restrict__ st) {
  final_sum<3>(partials, [&](const double* o) {
    if (st[T3_STOP] != 0.0) return;
    st[T3_ITER] += 1.0;
    st[T3_RR] = o[0];
    st[T3_RHO_NEW] = o[1];
    st[T3_RHO_NEW + 1] = o[2];
    if (o[0] <= st[T3_TOL2] * st[T3_BB] || st[T3_ITER] >= st[T3_MAXIT]) st[T3_STOP] = 1.0;
  });
}

template <int S>
hipError_t init_impl(const Trap3Bufs& b, const double* vraw, int64_t npts, double tau,
                     double tol2, int max_iter, hipStream_t st) {
  hipLaunchKernelGGL(k_t3_init<S>, dim3(kNB), dim3(kTB), 0, st, (const cd_t*)b.qz,
                     (const cd_t*)b.qy, (const cd_t*)b.qx, (const cd_t*)b.x, vraw, npts, tau,
                     (cd_t*)b.r, (cd_t*)b.p, b.partials);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_t3_final_init, dim3(1), dim3(kTB), 0, st, b.partials, tol2, max_iter,
                     b.sums);
  return hipGetLastError();
}

template <int S>
hipError_t ap_impl(const Trap3Bufs& b, const double* vraw, int64_t npts, double tau,
                   hipStream_t st) {
  hipLaunchKernelGGL(k_t3_ap<S>, dim3(kNB), dim3(kTB), 0, st, (const cd_t*)b.qz,
                     (const cd_t*)b.qy, (const cd_t*)b.qx, (const cd_t*)b.p, vraw, npts, tau,
                     (cd_t*)b.ap, b.partials);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_t3_final_ap, dim3(1), dim3(kTB), 0, st, b.partials, b.sums);
  return hipGetLastError();
}

}  // namespace

hipError_t t3_init(const Trap3Bufs& b, int S, const double* vraw, int64_t npts, double tau,
                   double tol2, int max_iter, hipStream_t st) {
  switch (S) {
    case 1: return init_impl<1>(b, vraw, npts, tau, tol2, max_iter, st);
    case 2: return init_impl<2>(b, vraw, npts, tau, tol2, max_iter, st);
    case 3: return init_impl<3>(b, vraw, npts, tau, tol2, max_iter, st);
    default: return hipErrorInvalidValue;
  }
}

hipError_t t3_ap(const Trap3Bufs& b, int S, const double* vraw, int64_t npts, double tau,
                 hipStream_t st) {
  switch (S) {
    case 1: return ap_impl<1>(b, vraw, npts, tau, st);
    case 2: return ap_impl<2>(b, vraw, npts, tau, st);
    case 3: return ap_impl<3>(b, vraw, npts, tau, st);
    default: return hipErrorInvalidValue;
  }
}

hipError_t t3_update(const Trap3Bufs& b, int64_t n, hipStream_t st) {
  hipLaunchKernelGGL(k_t3_update, dim3(kNB), dim3(kTB), 0, st, (cd_t*)b.x, (cd_t*)b.r,
                     (const cd_t*)b.p, (const cd_t*)b.ap, n, (const double*)b.sums, b.partials);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_t3_final_update, dim3(1), dim3(kTB), 0, st, b.partials, b.sums);
  return hipGetLastError();
}

hipError_t t3_pupdate(const Trap3Bufs& b, int64_t n, hipStream_t st) {
  hipLaunchKernelGGL(k_t3_pupdate, dim3(kNB), dim3(kTB), 0, st, (const cd_t*)b.r, (cd_t*)b.p, n,
                     (const double*)b.sums);
  return hipGetLastError();
}

}  // namespace sop
