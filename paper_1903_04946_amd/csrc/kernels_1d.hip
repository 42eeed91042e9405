// kernels_1d.hip -- one-dimensional grids: the whole composed time step runs
// inside one persistent workgroup per wavepacket.
//
// The S-surface state stays in registers (radix-R_first ownership) for all
// nsteps x (N_A + N_B) actions of the pruned sequence (Sec. "Pruning
// splitting coefficients"); only the FFT stage exchanges touch LDS, and HBM
// sees psi at entry and exit.  A potential action is the S x S matvec with
// the stored table exp(-i a dt V(x)/hbar) of its unique coefficient
// (Eq. range_index_unq); a kinetic action is forward FFT -> phase (with 1/N
// folded in) -> inverse FFT (Sec. "Dynamic Fourier method").  A direction of
// -1 conjugates every table, which is U(-dt).
#include "fft_core.hpp"
#include "internal.hpp"

namespace sop {
namespace {

// schedules: (N, E, forward radices, inverse radices = reversed, first, last).
// Eight values per thread and surface keep a two-surface FP64 state plus a
// radix-8 butterfly in about 128 VGPRs.
using S16 = Sched<16, 4, RList<4, 4>, RList<4, 4>, 4, 4>;
using S32 = Sched<32, 8, RList<8, 4>, RList<4, 8>, 8, 4>;
using S64 = Sched<64, 8, RList<8, 8>, RList<8, 8>, 8, 8>;
using S128 = Sched<128, 8, RList<8, 4, 4>, RList<4, 4, 8>, 8, 4>;
using S256 = Sched<256, 8, RList<8, 8, 4>, RList<4, 8, 8>, 8, 4>;
using S512 = Sched<512, 8, RList<8, 8, 8>, RList<8, 8, 8>, 8, 8>;
using S1024 = Sched<1024, 8, RList<8, 4, 4, 8>, RList<8, 4, 4, 8>, 8, 8>;
using S2048 = Sched<2048, 8, RList<8, 8, 4, 8>, RList<8, 4, 8, 8>, 8, 8>;
using S4096 = Sched<4096, 8, RList<8, 8, 8, 8>, RList<8, 8, 8, 8>, 8, 8>;
using S8192 = Sched<8192, 8, RList<8, 8, 8, 8, 2>, RList<2, 8, 8, 8, 8>, 8, 2>;

template <class SC>
constexpr int lds_pencil() {
  return SC::N + SC::N / 16;
}

// PL = pencils exchanged through LDS at once (S, or 1 when S pencils do not fit).
template <typename T, class SC, int S, int PL>
__global__ void __launch_bounds__(SC::TPC)
    k1d_prop_kernel(cx<T>* __restrict__ psi, const cx<T>* __restrict__ vexp,
                    const cx<T>* __restrict__ kin, const cx<T>* __restrict__ tw,
                    const int* __restrict__ prog, int nact, int64_t nsteps, int conj) {
  extern __shared__ char smem_raw[];
  cx<T>* lds = reinterpret_cast<cx<T>*>(smem_raw);
  constexpr int N = SC::N, E = SC::E, NE = S * (S + 1) / 2;
  const int t = threadIdx.x;
  psi += (size_t)blockIdx.x * S * N;  // one workgroup per state
  const T csign = conj ? (T)-1 : (T)1;
  cx<T> v[S][E];
#pragma unroll
  for (int s = 0; s < S; ++s)
#pragma unroll
    for (int q = 0; q < E; ++q) v[s][q] = psi[s * N + own_idx<N, E, SC::RF>(t, q)];
  const LayPadded lay{0, lds_pencil<SC>()};

  for (int64_t step = 0; step < nsteps; ++step) {
    for (int a = 0; a < nact; ++a) {
      const int code = prog[a];
      const int idx = code & 0xffff;
      if ((code >> 16) == OP_V) {
        const cx<T>* U = vexp + (size_t)idx * NE * N;
#pragma unroll
        for (int q = 0; q < E; ++q) {
          const int x = own_idx<N, E, SC::RF>(t, q);
          cx<T> u[NE];
#pragma unroll
          for (int e = 0; e < NE; ++e) {
            u[e] = U[e * N + x];
            u[e].im *= csign;
          }
          cx<T> w[S];
#pragma unroll
          for (int s = 0; s < S; ++s) w[s] = v[s][q];
          apply_u<T, S>(w, u);
#pragma unroll
          for (int s = 0; s < S; ++s) v[s][q] = w[s];
        }
      } else {
        if constexpr (PL == S) {
          fft_forward<SC, S>(v, lds, lay, tw, t);
        } else {
#pragma unroll
          for (int s = 0; s < S; ++s) fft_forward<SC, 1>(v + s, lds, lay, tw, t);
        }
        const cx<T>* F = kin + (size_t)idx * N;
#pragma unroll
        for (int q = 0; q < E; ++q) {
          cx<T> f = F[own_idx<N, E, SC::RL>(t, q)];
          f.im *= csign;
#pragma unroll
          for (int s = 0; s < S; ++s) v[s][q] = cmul(v[s][q], f);
        }
        if constexpr (PL == S) {
          fft_inverse<SC, S>(v, lds, lay, tw, t);
        } else {
#pragma unroll
          for (int s = 0; s < S; ++s) fft_inverse<SC, 1>(v + s, lds, lay, tw, t);
        }
      }
    }
  }
#pragma unroll
  for (int s = 0; s < S; ++s)
#pragma unroll
    for (int q = 0; q < E; ++q) psi[s * N + own_idx<N, E, SC::RF>(t, q)] = v[s][q];
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
  if (one * S <= kMaxLds) {
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
  return dispatch(d.n[0], d.S, d.f64, [&]<typename T, class SC, int S>() {
    return launch_prop<T, SC, S>(d, psi, nsteps, conj, count);
  });
}

hipError_t k1d_fft_forward(const DevView& d, void* psi) {
  return dispatch(d.n[0], d.S, d.f64, [&]<typename T, class SC, int S>() {
    return launch_fft<T, SC, S>(d, psi);
  });
}

}  // namespace sop
