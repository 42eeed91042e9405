// kernels_1d.hip -- one-dimensional grids: the whole composed time step runs
// inside one persistent workgroup per wavepacket (the step body is run_1d).
#include "body_1d.hpp"
#include "body_1d_w4.hpp"

namespace sop {
namespace {

using namespace s1d;

// PL = pencils exchanged through LDS at once (S, or 1 when S pencils do not fit).
template <typename T, class SC, int S, int PL>
__global__ void __launch_bounds__(SC::TPC)
    k1d_prop_kernel(cx<T>* __restrict__ psi, const cx<T>* __restrict__ vexp,
                    const cx<T>* __restrict__ kin, const cx<T>* __restrict__ tw,
                    const int* __restrict__ prog, int nact, int64_t nsteps, int conj) {
  extern __shared__ char smem_raw[];
  cx<T>* lds = reinterpret_cast<cx<T>*>(smem_raw);
  psi += (size_t)blockIdx.x * S * SC::N;  // one workgroup per state
  run_1d<T, SC, S, PL>(psi, vexp, kin, tw, prog, nact, nsteps, conj, lds);
}

// Two surfaces of 1024 points: the four-wave body.
template <typename T>
__global__ void __launch_bounds__(w4::kThreads)
    k1d_w4_kernel(cx<T>* __restrict__ psi, const cx<T>* __restrict__ vexp,
                  const cx<T>* __restrict__ kin, const cx<T>* __restrict__ tw,
                  const int* __restrict__ prog, int nact, int64_t nsteps, int conj) {
  extern __shared__ char smem_raw[];
  cx<T>* lds = reinterpret_cast<cx<T>*>(smem_raw);
  psi += (size_t)blockIdx.x * 2 * w4::N;  // one workgroup per state
  run_1d_w4<T>(psi, vexp, kin, tw, prog, nact, nsteps, conj, lds);
}

// Forward transform of every surface (natural order in and out), used for
// the kinetic energy.
template <typename T, class SC, int S>
__global__ void __launch_bounds__(SC::TPC)
    k1d_fft_kernel(cx<T>* __restrict__ psi, const cx<T>* __restrict__ tw) {
  extern __shared__ char smem_raw[];
  cx<T>* lds = reinterpret_cast<cx<T>*>(smem_raw);
  constexpr int N = SC::N, E = SC::E;
  const int t = threadIdx.x;
  cx<T> v[1][E];
  const LayPadded lay{0, lds_pencil<SC>()};
  for (int s = 0; s < S; ++s) {
#pragma unroll
    for (int q = 0; q < E; ++q) v[0][q] = psi[s * N + own_idx<N, E, SC::RF>(t, q)];
    fft_forward<SC, 1>(v, lds, lay, tw, t);
#pragma unroll
    for (int q = 0; q < E; ++q) psi[s * N + own_idx<N, E, SC::RL>(t, q)] = v[0][q];
  }
}

constexpr size_t kMaxLds = 160 * 1024;

template <typename T, class SC, int S>
hipError_t launch_prop(const DevView& d, void* psi, int64_t nsteps, int conj, int count) {
  constexpr size_t one = (size_t)lds_pencil<SC>() * sizeof(cx<T>);
  TimedLaunch tl(d, KIND_1D, 2.0 * S * SC::N * sizeof(cx<T>) * count);
  if constexpr (SC::N == w4::N && S == 2) {
    constexpr size_t bytes = w4::lds_bytes<T>();
    auto k = k1d_w4_kernel<T>;
    hipError_t e = hipFuncSetAttribute((const void*)k, hipFuncAttributeMaxDynamicSharedMemorySize,
                                       (int)bytes);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k, dim3(count), dim3(w4::kThreads), bytes, d.stream, (cx<T>*)psi,
                       (const cx<T>*)d.vexp, (const cx<T>*)d.kin, (const cx<T>*)d.tw[0], d.prog,
                       d.nact, nsteps, conj);
  } else if (one * S <= kMaxLds) {
    auto k = k1d_prop_kernel<T, SC, S, S>;
    hipError_t e = hipFuncSetAttribute((const void*)k, hipFuncAttributeMaxDynamicSharedMemorySize,
                                       (int)(one * S));
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k, dim3(count), dim3(SC::TPC), one * S, d.stream, (cx<T>*)psi,
                       (const cx<T>*)d.vexp, (const cx<T>*)d.kin, (const cx<T>*)d.tw[0], d.prog,
                       d.nact, nsteps, conj);
  } else {
    auto k = k1d_prop_kernel<T, SC, S, 1>;
    hipError_t e = hipFuncSetAttribute((const void*)k, hipFuncAttributeMaxDynamicSharedMemorySize,
                                       (int)one);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k, dim3(count), dim3(SC::TPC), one, d.stream, (cx<T>*)psi,
                       (const cx<T>*)d.vexp, (const cx<T>*)d.kin, (const cx<T>*)d.tw[0], d.prog,
                       d.nact, nsteps, conj);
  }
  return hipGetLastError();
}

template <typename T, class SC, int S>
hipError_t launch_fft(const DevView& d, void* psi) {
  constexpr size_t one = (size_t)lds_pencil<SC>() * sizeof(cx<T>);
  auto k = k1d_fft_kernel<T, SC, S>;
  hipError_t e =
      hipFuncSetAttribute((const void*)k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)one);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k, dim3(1), dim3(SC::TPC), one, d.stream, (cx<T>*)psi,
                     (const cx<T>*)d.tw[0]);
  return hipGetLastError();
}

template <class F>
hipError_t dispatch(int n, int S, bool f64, F&& f) {
#define SOP_1D_CASE(NN)                                                        \
  case NN:                                                                     \
    if (f64) {                                                                 \
      if (S == 1) return f.template operator()<double, S##NN, 1>();            \
      if (S == 2) return f.template operator()<double, S##NN, 2>();            \
    } else {                                                                   \
      if (S == 1) return f.template operator()<float, S##NN, 1>();             \
      if (S == 2) return f.template operator()<float, S##NN, 2>();             \
    }                                                                          \
    return hipErrorInvalidValue;
  switch (n) {
    SOP_1D_CASE(16)
    SOP_1D_CASE(32)
    SOP_1D_CASE(64)
    SOP_1D_CASE(128)
    SOP_1D_CASE(256)
    SOP_1D_CASE(512)
    SOP_1D_CASE(1024)
    SOP_1D_CASE(2048)
    SOP_1D_CASE(4096)
    SOP_1D_CASE(8192)
    default:
      return hipErrorInvalidValue;
  }
#undef SOP_1D_CASE
}

}  // namespace

bool k1d_supported(int n, int S) {
  if (S < 1 || S > 2) return false;
  switch (n) {
    case 16: case 32: case 64: case 128: case 256: case 512:
    case 1024: case 2048: case 4096: case 8192:
      return true;
    default:
      return false;
  }
}

hipError_t k1d_propagate(const DevView& d, void* psi, int64_t nsteps, int conj, int count) {
  if (d.timer) d.timer->break_chain();  // untimed work may precede this call
  return dispatch(d.n[0], d.S, d.f64, [&]<typename T, class SC, int S>() {
    return launch_prop<T, SC, S>(d, psi, nsteps, conj, count);
  });
}

hipError_t k1d_fft_forward(const DevView& d, void* psi) {
  if (d.timer) d.timer->break_chain();  // untimed work may precede this call
  return dispatch(d.n[0], d.S, d.f64, [&]<typename T, class SC, int S>() {
    return launch_fft<T, SC, S>(d, psi);
  });
}

}  // namespace sop
