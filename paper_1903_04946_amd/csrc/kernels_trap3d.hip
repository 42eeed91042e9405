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

// x += alpha p, r -= alpha ap.  Partials: |r|^2, r^T r (re, im).
__global__ void __launch_bounds__(kTB)
    k_t3_update(cd_t* __restrict__ x, cd_t* __restrict__ r, const cd_t* __restrict__ p,
                const cd_t* __restrict__ ap, int64_t n, double are, double aim,
                double* __restrict__ partials) {
  const cd_t alpha = {are, aim};
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

// p = r + beta p.
__global__ void __launch_bounds__(kTB)
    k_t3_pupdate(const cd_t* __restrict__ r, cd_t* __restrict__ p, int64_t n, double bre,
                 double bim) {
  const cd_t beta = {bre, bim};
  for (int64_t i = (int64_t)blockIdx.x * kTB + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * kTB)
    p[i] = cadd(r[i], cmul(beta, p[i]));
}

// out[v] = sum over the kNB blocks of partials[b][v], in a fixed order.
__global__ void __launch_bounds__(kTB)
    k_t3_final(const double* __restrict__ partials, int nv, double* __restrict__ out) {
  __shared__ double red[kTB];
  for (int v = 0; v < nv; ++v) {
    double acc = 0.0;
    for (int b = threadIdx.x; b < kNB; b += kTB) acc += partials[(size_t)b * nv + v];
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int w = kTB / 2; w > 0; w >>= 1) {
      if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
      __syncthreads();
    }
    if (threadIdx.x == 0) out[v] = red[0];
    __syncthreads();
  }
}

template <int S>
hipError_t init_impl(const Trap3Bufs& b, const double* vraw, int64_t npts, double tau,
                     hipStream_t st) {
  hipLaunchKernelGGL(k_t3_init<S>, dim3(kNB), dim3(kTB), 0, st, (const cd_t*)b.qz,
                     (const cd_t*)b.qy, (const cd_t*)b.qx, (const cd_t*)b.x, vraw, npts, tau,
                     (cd_t*)b.r, (cd_t*)b.p, b.partials);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_t3_final, dim3(1), dim3(kTB), 0, st, b.partials, 4, b.sums);
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
  hipLaunchKernelGGL(k_t3_final, dim3(1), dim3(kTB), 0, st, b.partials, 2, b.sums);
  return hipGetLastError();
}

}  // namespace

hipError_t t3_init(const Trap3Bufs& b, int S, const double* vraw, int64_t npts, double tau,
                   hipStream_t st) {
  switch (S) {
    case 1: return init_impl<1>(b, vraw, npts, tau, st);
    case 2: return init_impl<2>(b, vraw, npts, tau, st);
    case 3: return init_impl<3>(b, vraw, npts, tau, st);
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

hipError_t t3_update(const Trap3Bufs& b, int64_t n, double are, double aim, hipStream_t st) {
  hipLaunchKernelGGL(k_t3_update, dim3(kNB), dim3(kTB), 0, st, (cd_t*)b.x, (cd_t*)b.r,
                     (const cd_t*)b.p, (const cd_t*)b.ap, n, are, aim, b.partials);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_t3_final, dim3(1), dim3(kTB), 0, st, b.partials, 3, b.sums);
  return hipGetLastError();
}

hipError_t t3_pupdate(const Trap3Bufs& b, int64_t n, double bre, double bim, hipStream_t st) {
  hipLaunchKernelGGL(k_t3_pupdate, dim3(kNB), dim3(kTB), 0, st, (const cd_t*)b.r, (cd_t*)b.p, n,
                     bre, bim);
  return hipGetLastError();
}

}  // namespace sop
