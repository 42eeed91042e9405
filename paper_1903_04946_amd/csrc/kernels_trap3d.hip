// kernels_trap3d.hip -- pointwise and reduction kernels of the trapezoidal
// rule on 3D grids (FP64).
//
// A stage of the trapezoidal rule solves (1 + i tau H) x = (1 - i tau H) psi
// with the conjugate orthogonal conjugate gradient method (H is real
// symmetric on the grid, so 1 + i tau H is complex symmetric).  On a 3D grid
// the kinetic part of H p is the sum of three one-axis terms,
// T p = sum_d F_d^-1 T_d(k) F_d p, each computed by a pass kernel of the
// propagator that reads p and writes its own term, with the factor
// T_d(k)/n_d in place of the phase (the host sequences them); the kernels
// here add the three terms and the S x S matvec with V(x), form
// A p = p + i tau H p, update the iterates, and reduce the inner products
// the method needs (u^T v without conjugation, and |u|^2) in a fixed order:
// block partials, then a tree over the blocks.
//
// The iteration's scalars stay on the device.  Each block of the update
// kernels forms mu, rho and |r|^2 from the partials itself, every block in
// the same order, so no separate reduction kernel runs; the residual
// partials of consecutive iterations alternate between two buffers (by the
// iteration's parity) so that a kernel reads the previous ones while it
// writes the new ones.  Block 0 keeps the status block (T3_*: iteration
// count, |r|^2, stop and breakdown flags), which the host reads every few
// iterations.  Once the residual test holds (or mu breaks down, or the
// iteration limit is reached) the status freezes the iterate: later
// iterations use alpha = beta = 0 and leave x unchanged.
#include "fft_core.hpp"
#include "internal.hpp"

namespace sop {
namespace {

typedef cx<double> cd_t;

constexpr int kTB = kReduceThreads;  // threads per block
constexpr int kNB = kReduceBlocks;   // most blocks (grid-stride over the points)

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
// -2 i tau h, p = r.  Partials: |b|^2 into pb, and |r|^2, r^T r (re, im)
// into pu (the residual partials of "iteration -1").
template <int S>
__global__ void __launch_bounds__(kTB)
    k_t3_init(const cd_t* __restrict__ qz, const cd_t* __restrict__ qy,
              const cd_t* __restrict__ qx, const cd_t* __restrict__ x,
              const double* __restrict__ vraw, int64_t npts, double tau, cd_t* __restrict__ r,
              cd_t* __restrict__ p, double* __restrict__ pb, double* __restrict__ pu) {
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
  __shared__ double o[4];
  tsum<4>(acc, o);
  if (threadIdx.x == 0) {
    pb[blockIdx.x] = o[0];
    for (int v = 0; v < 3; ++v) pu[(size_t)blockIdx.x * 3 + v] = o[1 + v];
  }
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

__device__ __forceinline__ cd_t cdiv(double are, double aim, double bre, double bim) {
  const double den = bre * bre + bim * bim;
  return {(are * bre + aim * bim) / den, (aim * bre - are * bim) / den};
}

// Every block's copy of out[v] = sum over b < nb of partials[b][v], in the
// same fixed order in every block (strided per thread, then a tree).
template <int NV>
__device__ void block_total(const double* __restrict__ partials, int nb, double (&out)[NV]) {
  double acc[NV];
#pragma unroll
  for (int v = 0; v < NV; ++v) acc[v] = 0.0;
  for (int b = threadIdx.x; b < nb; b += kTB) {
#pragma unroll
    for (int v = 0; v < NV; ++v) acc[v] += partials[(size_t)b * NV + v];
  }
  __shared__ double sh[NV];
  tsum<NV>(acc, sh);
  __syncthreads();
#pragma unroll
  for (int v = 0; v < NV; ++v) out[v] = sh[v];
}

// x += alpha p, r -= alpha ap.  Every block forms mu = p^T A p from the
// A p partials pa and rho = r^T r from the previous residual partials
// pu_prev (no separate reduction kernel), alpha = rho / mu, or 0 if the
// status is frozen or mu breaks down.  Partials of the new residual: |r|^2,
// r^T r (re, im) into pu_cur.  Block 0 counts the iteration (or records the
// breakdown) in the status; the other blocks reach the same decision from
// the same sums.
template <int S>
__global__ void __launch_bounds__(kTB)
    k_t3_update(cd_t* __restrict__ x, cd_t* __restrict__ r, const cd_t* __restrict__ p,
                const cd_t* __restrict__ ap, int64_t npts, double* __restrict__ st,
                const double* __restrict__ pa, const double* __restrict__ pu_prev,
                double* __restrict__ pu_cur) {
  double mu[2], rho[3];
  block_total<2>(pa, gridDim.x, mu);
  block_total<3>(pu_prev, gridDim.x, rho);
  const bool stop0 = st[T3_STOP] != 0.0;
  const double mabs = fabs(mu[0]) + fabs(mu[1]);
  const bool breakdown = !(mabs > 0.0) || !(mabs < 1e300);
  const cd_t alpha = (stop0 || breakdown) ? cd_t{0.0, 0.0} : cdiv(rho[1], rho[2], mu[0], mu[1]);
  double acc[3] = {0.0, 0.0, 0.0};
  for (int64_t k = (int64_t)blockIdx.x * kTB + threadIdx.x; k < npts;
       k += (int64_t)gridDim.x * kTB) {
#pragma unroll
    for (int s = 0; s < S; ++s) {
      const int64_t i = s * npts + k;
      x[i] = cadd(x[i], cmul(alpha, p[i]));
      const cd_t rn = csub(r[i], cmul(alpha, ap[i]));
      r[i] = rn;
      acc[0] += rn.re * rn.re + rn.im * rn.im;
      acc[1] += rn.re * rn.re - rn.im * rn.im;
      acc[2] += 2.0 * rn.re * rn.im;
    }
  }
  tsum<3>(acc, pu_cur + (size_t)blockIdx.x * 3);
  if (blockIdx.x == 0 && threadIdx.x == 0 && !stop0) {
    if (breakdown) {
      st[T3_FAIL] = 1.0;
      st[T3_STOP] = 1.0;
    } else {
      st[T3_ITER] += 1.0;
      st[T3_MU] = mu[0];
      st[T3_MU + 1] = mu[1];
    }
  }
}

// p = r + beta p.  Every block forms |r|^2 and rho_new from the new residual
// partials pu_cur and rho from pu_prev: beta = rho_new / rho, or 0 once the
// residual test holds, the iteration limit is reached or the status is
// frozen.  Block 0 records |r|^2 and, when the test holds or the limit is
// reached, freezes the status.
__global__ void __launch_bounds__(kTB)
    k_t3_pupdate(const cd_t* __restrict__ r, cd_t* __restrict__ p, int64_t n,
                 double* __restrict__ st, const double* __restrict__ pu_prev,
                 const double* __restrict__ pu_cur, int nbu) {
  double cur[3], prev[3];
  block_total<3>(pu_cur, nbu, cur);
  block_total<3>(pu_prev, nbu, prev);
  const bool stop0 = st[T3_STOP] != 0.0;
  const bool conv = cur[0] <= st[T3_TOL2] * st[T3_BB] || st[T3_ITER] >= st[T3_MAXIT];
  const cd_t beta = (stop0 || conv) ? cd_t{0.0, 0.0} : cdiv(cur[1], cur[2], prev[1], prev[2]);
  for (int64_t i = (int64_t)blockIdx.x * kTB + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * kTB)
    p[i] = cadd(r[i], cmul(beta, p[i]));
  if (blockIdx.x == 0 && threadIdx.x == 0 && !stop0) {
    st[T3_RR] = cur[0];
    st[T3_RHO] = cur[1];
    st[T3_RHO + 1] = cur[2];
    if (conv) st[T3_STOP] = 1.0;
  }
}

// Blocks of a pass over n items: enough for one item per thread, at most kNB.
inline int nblocks(int64_t n) {
  const int64_t b = (n + kTB - 1) / kTB;
  return (int)(b < 1 ? 1 : (b > kNB ? kNB : b));
}

// Start of a stage: |b|^2, |r|^2 and rho = r^T r; converged at once if
// |r|^2 <= tol^2 |b|^2.
__global__ void __launch_bounds__(kTB)
    k_t3_final_init(const double* __restrict__ pb, const double* __restrict__ pu, int nb,
                    double tol2, int max_iter, double* __restrict__ st) {
  double bb[1], ru[3];
  block_total<1>(pb, nb, bb);
  block_total<3>(pu, nb, ru);
  if (threadIdx.x == 0) {
    st[T3_BB] = bb[0];
    st[T3_RR] = ru[0];
    st[T3_RHO] = ru[1];
    st[T3_RHO + 1] = ru[2];
    st[T3_TOL2] = tol2;
    st[T3_MAXIT] = (double)max_iter;
    st[T3_STOP] = ru[0] <= tol2 * bb[0] ? 1.0 : 0.0;
    st[T3_ITER] = 0.0;
    st[T3_FAIL] = 0.0;
  }
}

// Partial-sum buffers of the iteration (doubles, kNB blocks each): |b|^2,
// the A p partials, and the residual partials of the last two iterations
// (by parity; "iteration -1" is the start of the stage, parity 1).
struct Parts {
  double *pb, *pa, *pu[2];
  explicit Parts(double* base)
      : pb(base), pa(base + kNB), pu{base + 3 * kNB, base + 6 * kNB} {}
};

template <int S>
hipError_t init_impl(const Trap3Bufs& b, const double* vraw, int64_t npts, double tau,
                     double tol2, int max_iter, hipStream_t st) {
  const int nb = nblocks(npts);
  const Parts q(b.partials);
  hipLaunchKernelGGL(k_t3_init<S>, dim3(nb), dim3(kTB), 0, st, (const cd_t*)b.qz,
                     (const cd_t*)b.qy, (const cd_t*)b.qx, (const cd_t*)b.x, vraw, npts, tau,
                     (cd_t*)b.r, (cd_t*)b.p, q.pb, q.pu[1]);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_t3_final_init, dim3(1), dim3(kTB), 0, st, (const double*)q.pb,
                     (const double*)q.pu[1], nb, tol2, max_iter, b.sums);
  return hipGetLastError();
}

template <int S>
hipError_t ap_impl(const Trap3Bufs& b, const double* vraw, int64_t npts, double tau,
                   hipStream_t st) {
  const Parts q(b.partials);
  hipLaunchKernelGGL(k_t3_ap<S>, dim3(nblocks(npts)), dim3(kTB), 0, st, (const cd_t*)b.qz,
                     (const cd_t*)b.qy, (const cd_t*)b.qx, (const cd_t*)b.p, vraw, npts, tau,
                     (cd_t*)b.ap, q.pa);
  return hipGetLastError();
}

template <int S>
hipError_t update_impl(const Trap3Bufs& b, int64_t npts, int parity, hipStream_t st) {
  const Parts q(b.partials);
  hipLaunchKernelGGL(k_t3_update<S>, dim3(nblocks(npts)), dim3(kTB), 0, st, (cd_t*)b.x,
                     (cd_t*)b.r, (const cd_t*)b.p, (const cd_t*)b.ap, npts, b.sums,
                     (const double*)q.pa, (const double*)q.pu[1 - parity], q.pu[parity]);
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

hipError_t t3_update(const Trap3Bufs& b, int S, int64_t npts, int parity, hipStream_t st) {
  switch (S) {
    case 1: return update_impl<1>(b, npts, parity, st);
    case 2: return update_impl<2>(b, npts, parity, st);
    case 3: return update_impl<3>(b, npts, parity, st);
    default: return hipErrorInvalidValue;
  }
}

hipError_t t3_pupdate(const Trap3Bufs& b, int S, int64_t npts, int parity, hipStream_t st) {
  const Parts q(b.partials);
  hipLaunchKernelGGL(k_t3_pupdate, dim3(nblocks((int64_t)S * npts)), dim3(kTB), 0, st,
                     (const cd_t*)b.r, (cd_t*)b.p, (int64_t)S * npts, b.sums,
                     (const double*)q.pu[1 - parity], (const double*)q.pu[parity],
                     nblocks(npts));
  return hipGetLastError();
}

}  // namespace sop
