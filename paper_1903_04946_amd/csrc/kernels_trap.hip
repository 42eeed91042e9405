// kernels_trap.hip -- compositions of the trapezoidal rule on 1D grids.
//
// The trapezoidal rule (Crank-Nicolson; for a linear equation the same map as
// the implicit midpoint rule) advances i hbar dpsi/dt = H psi by
// (1 + i tau H) psi' = (1 - i tau H) psi, tau = g dt / (2 hbar): a symmetric,
// second-order, unitary and energy-conserving method, composed with the same
// coefficients g as the split-operator steps (Sec. "Symmetric composition
// schemes").  Each stage needs a linear solve.  H = T + V is real symmetric
// on the grid (T(k) even in k), so A = 1 + i tau H is complex symmetric and
// the conjugate orthogonal conjugate gradient method (CG with the bilinear
// form u^T v) solves it with two vectors in registers per thread; since
// |1 + i tau lambda| >= 1, the error of the solution is at most the residual.
//
// One workgroup holds one wavepacket for all its steps: H p is an FFT round
// trip through LDS with T(k)/N applied in between, plus the S x S matvec with
// V(x); the iterate x and the residual r live in global memory (each element
// touched only by the thread that owns it), the direction p and H p in
// registers; dot products are workgroup sums in a fixed order.  The loop
// ends for every thread together: its conditions are block-wide values.
#include <mutex>

#include "body_1d.hpp"

// Device scratch of sop_propagate_trapezoid_noalloc (residuals, per-state
// statistics, stage coefficients): a fixed array per GPU, held until the
// process ends, so that the call needs no allocation.  Host code never
// passes this name to a kernel or a copy: it is a host-side stand-in, and
// the device address comes from hipGetSymbolAddress (sop::trap_scratch).
static constexpr size_t kTrapScratchBytes = size_t(32) << 20;
static __device__ __align__(256) char scratch[kTrapScratchBytes];

namespace sop {
namespace {

using namespace s1d;

// Schedules of four values per thread (twice the threads of the propagation
// schedules, half the registers): the solver keeps two vectors in registers,
// and at eight values per thread it needs all 256 VGPRs, one wave per SIMD.
using T512 = Sched<512, 4, RList<4, 4, 4, 4, 2>, RList<2, 4, 4, 4, 4>, 4, 2>;
using T1024 = Sched<1024, 4, RList<4, 4, 4, 4, 4>, RList<4, 4, 4, 4, 4>, 4, 4>;
using T2048 = Sched<2048, 4, RList<4, 4, 4, 4, 4, 2>, RList<2, 4, 4, 4, 4, 4>, 4, 2>;
using T4096 = Sched<4096, 4, RList<4, 4, 4, 4, 4, 4>, RList<4, 4, 4, 4, 4, 4>, 4, 4>;
using T8192 = S8192;  // 1024 threads already
// At 1024 threads a wave gets at most 128 VGPRs, so the 4096- and 8192-point
// kernels spill (gfx950 build: 160 / 504 bytes per lane at 4096 points with
// one / two surfaces, 212 / 1592 at 8192); 512 threads of eight values per
// thread spill as much at 4096 points and two surfaces (460 bytes).

typedef cx<double> cd_t;

__device__ __forceinline__ cd_t cdiv(cd_t a, cd_t b) {
  const double den = b.re * b.re + b.im * b.im;
  return {(a.re * b.re + a.im * b.im) / den, (a.im * b.re - a.re * b.im) / den};
}

// Workgroup sums of K doubles (TPC a multiple of 64); every thread receives
// them.  The first barrier keeps a previous call's readers ahead of the writes.
template <int TPC, int K>
__device__ __forceinline__ void block_sum(double (&a)[K], double* red) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1)
#pragma unroll
    for (int k = 0; k < K; ++k) a[k] += __shfl_xor(a[k], off);
  constexpr int NW = TPC / 64;
  const int w = threadIdx.x / 64;
  __syncthreads();
  if (threadIdx.x % 64 == 0)
#pragma unroll
    for (int k = 0; k < K; ++k) red[K * w + k] = a[k];
  __syncthreads();
#pragma unroll
  for (int k = 0; k < K; ++k) {
    double s = 0.0;
    for (int i = 0; i < NW; ++i) s += red[K * i + k];
    a[k] = s;
  }
}

// v <- H p on the owned elements (RF layout).
template <class SC, int S, int PL>
__device__ __forceinline__ void apply_h(cd_t (&p)[S][SC::E], cd_t (&v)[S][SC::E], cd_t* lds,
                                        const cd_t* __restrict__ tw,
                                        const double* __restrict__ vraw, double tk, int t) {
  constexpr int N = SC::N, E = SC::E;
  const LayPadded lay{0, lds_pencil<SC>()};
#pragma unroll
  for (int s = 0; s < S; ++s)
#pragma unroll
    for (int q = 0; q < E; ++q) v[s][q] = p[s][q];
  if constexpr (PL == S) {
    fft_forward<SC, S>(v, lds, lay, tw, t);
  } else {
#pragma unroll
    for (int s = 0; s < S; ++s) fft_forward<SC, 1>(v + s, lds, lay, tw, t);
  }
#pragma unroll
  for (int q = 0; q < E; ++q) {
    const int k = own_idx<N, E, SC::RL>(t, q);
    const double ks = k <= N / 2 ? (double)k : (double)(k - N);
    const double f = tk * ks * ks / N;  // T(k), with the 1/N of the inverse transform
#pragma unroll
    for (int s = 0; s < S; ++s) v[s][q] = {v[s][q].re * f, v[s][q].im * f};
  }
  if constexpr (PL == S) {
    fft_inverse<SC, S>(v, lds, lay, tw, t);
  } else {
#pragma unroll
    for (int s = 0; s < S; ++s) fft_inverse<SC, 1>(v + s, lds, lay, tw, t);
  }
#pragma unroll
  for (int q = 0; q < E; ++q) {
    const int x = own_idx<N, E, SC::RF>(t, q);
#pragma unroll
    for (int s = 0; s < S; ++s)
#pragma unroll
      for (int r = 0; r < S; ++r) {
        const int a = s < r ? s : r, b = s < r ? r : s;
        const double vv = vraw[(size_t)(a * S - a * (a - 1) / 2 + (b - a)) * N + x];
        v[s][q].re = fma(vv, p[r][q].re, v[s][q].re);
        v[s][q].im = fma(vv, p[r][q].im, v[s][q].im);
      }
  }
}

// stats[3 * block] = {iterations, stages not converged, most iterations of a stage}.
template <class SC, int S, int PL>
__global__ void __launch_bounds__(SC::TPC) __attribute__((amdgpu_waves_per_eu(2)))
    k1d_trap_kernel(cd_t* __restrict__ psi, cd_t* __restrict__ rbuf,
                    const double* __restrict__ vraw, const cd_t* __restrict__ tw,
                    const double* __restrict__ taus, int nst, int64_t nsteps, double tk,
                    double tol2, int maxit, long long* __restrict__ stats) {
  extern __shared__ char smem_raw[];
  cd_t* lds = reinterpret_cast<cd_t*>(smem_raw);
  __shared__ double red[4 * (SC::TPC / 64)];
  constexpr int N = SC::N, E = SC::E;
  const int t = threadIdx.x;
  psi += (size_t)blockIdx.x * S * N;
  rbuf += (size_t)blockIdx.x * S * N;
  cd_t p[S][E], v[S][E];
  long long iters = 0, fails = 0;
  int worst = 0;
  for (int64_t step = 0; step < nsteps; ++step) {
    for (int j = 0; j < nst; ++j) {
      const double tau = taus[j];
#pragma unroll
      for (int s = 0; s < S; ++s)
#pragma unroll
        for (int q = 0; q < E; ++q) p[s][q] = psi[s * N + own_idx<N, E, SC::RF>(t, q)];
      apply_h<SC, S, PL>(p, v, lds, tw, vraw, tk, opaque(t));
      // b = psi - i tau H psi; with x0 = psi the residual is r0 = -2 i tau H psi
      double s4[4] = {0.0, 0.0, 0.0, 0.0};  // |b|^2, |r|^2, r^T r
#pragma unroll
      for (int s = 0; s < S; ++s)
#pragma unroll
        for (int q = 0; q < E; ++q) {
          const cd_t b = {p[s][q].re + tau * v[s][q].im, p[s][q].im - tau * v[s][q].re};
          const cd_t r = {2.0 * tau * v[s][q].im, -2.0 * tau * v[s][q].re};
          rbuf[s * N + own_idx<N, E, SC::RF>(t, q)] = r;
          s4[0] += b.re * b.re + b.im * b.im;
          s4[1] += r.re * r.re + r.im * r.im;
          s4[2] += r.re * r.re - r.im * r.im;
          s4[3] += 2.0 * r.re * r.im;
          p[s][q] = r;
        }
      block_sum<SC::TPC, 4>(s4, red);
      const double bb = s4[0];
      double rr = s4[1];
      cd_t rho = {s4[2], s4[3]};
      int it = 0;
      bool ok = rr <= tol2 * bb;
      while (!ok && it < maxit) {
        apply_h<SC, S, PL>(p, v, lds, tw, vraw, tk, opaque(t));
        double m2[2] = {0.0, 0.0};  // p^T A p
#pragma unroll
        for (int s = 0; s < S; ++s)
#pragma unroll
          for (int q = 0; q < E; ++q) {
            const cd_t aq = {p[s][q].re - tau * v[s][q].im, p[s][q].im + tau * v[s][q].re};
            v[s][q] = aq;
            m2[0] += p[s][q].re * aq.re - p[s][q].im * aq.im;
            m2[1] += p[s][q].re * aq.im + p[s][q].im * aq.re;
          }
        block_sum<SC::TPC, 2>(m2, red);
        const cd_t mu = {m2[0], m2[1]};
        const double mabs = fabs(mu.re) + fabs(mu.im);
        if (!(mabs > 0.0) || !(mabs < 1e300)) break;  // breakdown: reported as not converged
        const cd_t alpha = cdiv(rho, mu);
        double s3[3] = {0.0, 0.0, 0.0};
#pragma unroll
        for (int s = 0; s < S; ++s)
#pragma unroll
          for (int q = 0; q < E; ++q) {
            const int idx = s * N + own_idx<N, E, SC::RF>(t, q);
            psi[idx] = cadd(psi[idx], cmul(alpha, p[s][q]));
            const cd_t rn = csub(rbuf[idx], cmul(alpha, v[s][q]));
            rbuf[idx] = rn;
            v[s][q] = rn;
            s3[0] += rn.re * rn.re + rn.im * rn.im;
            s3[1] += rn.re * rn.re - rn.im * rn.im;
            s3[2] += 2.0 * rn.re * rn.im;
          }
        block_sum<SC::TPC, 3>(s3, red);
        ++it;
        rr = s3[0];
        ok = rr <= tol2 * bb;
        if (!ok) {
          const cd_t rhon = {s3[1], s3[2]};
          const cd_t beta = cdiv(rhon, rho);
          rho = rhon;
#pragma unroll
          for (int s = 0; s < S; ++s)
#pragma unroll
            for (int q = 0; q < E; ++q) p[s][q] = cadd(v[s][q], cmul(beta, p[s][q]));
        }
      }
      iters += it;
      worst = it > worst ? it : worst;
      if (!ok) ++fails;
    }
  }
  if (t == 0) {
    stats[3 * blockIdx.x] = iters;
    stats[3 * blockIdx.x + 1] = fails;
    stats[3 * blockIdx.x + 2] = worst;
  }
}

constexpr size_t kMaxLds = 160 * 1024;

template <class SC, int S>
hipError_t launch_trap(const DevView& d, const TrapArgs& g) {
  constexpr size_t one = (size_t)lds_pencil<SC>() * sizeof(cd_t);
  constexpr int PL = one * S <= kMaxLds ? S : 1;
  auto k = k1d_trap_kernel<SC, S, PL>;
  hipError_t e = hipFuncSetAttribute((const void*)k, hipFuncAttributeMaxDynamicSharedMemorySize,
                                     (int)(one * PL));
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k, dim3(g.count), dim3(SC::TPC), one * PL, d.stream, (cd_t*)g.psi,
                     (cd_t*)g.rbuf, g.vraw, (const cd_t*)d.tw[0], g.taus, g.nst, g.nsteps, g.tk,
                     g.tol2, g.maxit, g.stats);
  return hipGetLastError();
}

}  // namespace

size_t trap_scratch_bytes() { return kTrapScratchBytes; }

hipError_t trap_scratch(hipStream_t stream, void** out) {
  constexpr int kMaxDevices = 64;
  static std::mutex mu;
  static void* ptrs[kMaxDevices] = {};
  int dev = -1;
  hipError_t e = stream ? hipStreamGetDevice(stream, &dev) : hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(mu);
  if (!ptrs[dev]) {
    // once per device, with that device current: every GPU holds its own
    // copy of the array at its own address
    int cur = -1;
    e = hipGetDevice(&cur);
    if (e != hipSuccess) return e;
    if (cur != dev && (e = hipSetDevice(dev)) != hipSuccess) return e;
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (cur != dev) {
      const hipError_t r = hipSetDevice(cur);
      if (e == hipSuccess) e = r;
    }
    if (e != hipSuccess) return e;
    if (!p) return hipErrorInvalidSymbol;
    ptrs[dev] = p;
  }
  *out = ptrs[dev];
  return hipSuccess;
}

bool k1d_trap_supported(int n, int S) {
  return (S == 1 || S == 2) && (n == 512 || n == 1024 || n == 2048 || n == 4096 || n == 8192);
}

hipError_t k1d_trapezoid(const DevView& d, const TrapArgs& g) {
  if (!d.f64 || g.count < 1 || !k1d_trap_supported(d.n[0], d.S)) return hipErrorInvalidValue;
#define SOP_TRAP_CASE(NN)                                      \
  case NN:                                                     \
    return d.S == 1 ? launch_trap<T##NN, 1>(d, g) : launch_trap<T##NN, 2>(d, g);
  switch (d.n[0]) {
    SOP_TRAP_CASE(512)
    SOP_TRAP_CASE(1024)
    SOP_TRAP_CASE(2048)
    SOP_TRAP_CASE(4096)
    SOP_TRAP_CASE(8192)
    default:
      return hipErrorInvalidValue;
  }
#undef SOP_TRAP_CASE
}

}  // namespace sop
