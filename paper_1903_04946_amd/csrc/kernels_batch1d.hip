// kernels_batch1d.hip -- one-dimensional members of a batch: one launch per
// (grid length, surfaces, precision) family, one workgroup per member for
// its whole run (the composed step body run_1d, state in registers).
//
// Members are laid out in decreasing order of work, so the hardware
// dispatcher hands the longest runs out first and shorter ones fill the
// compute units as workgroups retire.  Each member has its own tables,
// program, step count and direction; the family only fixes the kernel.
//
// The schedule of a family (values per thread E, the radix sequence, and
// whether twiddles are recomputed per transform) is picked by the planner's
// tuner among the variants below; variant 0 is the schedule of the
// single-plan kernel.  All variants compute the same DFTs, in different
// radix orders.
#include "body_1d.hpp"
#include "body_1d_w4.hpp"

namespace sop {
namespace {

// alternative schedules: four and sixteen values per thread
template <int N>
struct Alt;
template <>
struct Alt<512> {
  using E4 = Sched<512, 4, RList<4, 4, 4, 4, 2>, RList<2, 4, 4, 4, 4>, 4, 2>;
  using E16 = Sched<512, 16, RList<16, 8, 4>, RList<4, 8, 16>, 16, 4>;
};
template <>
struct Alt<1024> {
  using E4 = Sched<1024, 4, RList<4, 4, 4, 4, 4>, RList<4, 4, 4, 4, 4>, 4, 4>;
  using E16 = Sched<1024, 16, RList<16, 16, 4>, RList<4, 16, 16>, 16, 4>;
};
template <>
struct Alt<2048> {
  using E4 = Sched<2048, 4, RList<4, 4, 4, 4, 4, 2>, RList<2, 4, 4, 4, 4, 4>, 4, 2>;
  using E16 = Sched<2048, 16, RList<16, 16, 8>, RList<8, 16, 16>, 16, 8>;
};
template <>
struct Alt<4096> {
  using E4 = Sched<4096, 4, RList<4, 4, 4, 4, 4, 4>, RList<4, 4, 4, 4, 4, 4>, 4, 4>;
  using E16 = Sched<4096, 16, RList<16, 16, 16>, RList<16, 16, 16>, 16, 16>;
};
template <>
struct Alt<8192> {
  using E16 = Sched<8192, 16, RList<8, 8, 8, 16>, RList<16, 8, 8, 8>, 8, 16>;
};

constexpr size_t kMaxLds = 160 * 1024;

template <typename T, class SC, int S, int PL, bool G>
__global__ void __launch_bounds__(SC::TPC)
    k1b_kernel(const BMember1* __restrict__ mem) {
  extern __shared__ char smem_raw[];
  cx<T>* lds = reinterpret_cast<cx<T>*>(smem_raw);
  const BMember1 m = mem[blockIdx.x];
  if (m.nsteps <= 0) return;
  run_1d<T, SC, S, PL, G>((cx<T>*)m.psi, (const cx<T>*)m.vexp, (const cx<T>*)m.kin,
                          (const cx<T>*)m.tw, m.prog, m.nact, m.nsteps, m.conj, lds);
}

template <typename T>
__global__ void __launch_bounds__(w4::kThreads) k1b_w4_kernel(const BMember1* __restrict__ mem) {
  extern __shared__ char smem_raw[];
  cx<T>* lds = reinterpret_cast<cx<T>*>(smem_raw);
  const BMember1 m = mem[blockIdx.x];
  if (m.nsteps <= 0) return;
  run_1d_w4<T>((cx<T>*)m.psi, (const cx<T>*)m.vexp, (const cx<T>*)m.kin, (const cx<T>*)m.tw,
               m.prog, m.nact, m.nsteps, m.conj, lds);
}

// two surfaces of 1024 points on four waves
hipError_t launch_w4(bool f64, const BMember1* mem, int count, hipStream_t stream) {
  auto go = [&](auto k, size_t bytes) {
    hipError_t e = hipFuncSetAttribute((const void*)k, hipFuncAttributeMaxDynamicSharedMemorySize,
                                       (int)bytes);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k, dim3(count), dim3(w4::kThreads), bytes, stream, mem);
    return hipGetLastError();
  };
  if (f64) return go(k1b_w4_kernel<double>, w4::lds_bytes<double>());
  return go(k1b_w4_kernel<float>, w4::lds_bytes<float>());
}

template <typename T, class SC, int S, bool G>
hipError_t launch(const BMember1* mem, int count, hipStream_t stream) {
  constexpr size_t one = (size_t)lds_pencil<SC>() * sizeof(cx<T>);
  if constexpr (one * S <= kMaxLds) {
    auto k = k1b_kernel<T, SC, S, S, G>;
    hipError_t e = hipFuncSetAttribute((const void*)k, hipFuncAttributeMaxDynamicSharedMemorySize,
                                       (int)(one * S));
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k, dim3(count), dim3(SC::TPC), one * S, stream, mem);
  } else {
    auto k = k1b_kernel<T, SC, S, 1, G>;
    hipError_t e = hipFuncSetAttribute((const void*)k, hipFuncAttributeMaxDynamicSharedMemorySize,
                                       (int)one);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k, dim3(count), dim3(SC::TPC), one, stream, mem);
  }
  return hipGetLastError();
}

// twiddle policy of a variant: the single-plan default of the precision,
// its opposite, or recomputed twiddles
enum { G_DEFAULT = 0, G_OTHER = 1, G_ON = 2 };
template <typename T, int N, int GM>
constexpr bool guard_of() {
  return GM == G_ON ? true : (GM == G_DEFAULT ? guard_default<T>(N) : !guard_default<T>(N));
}

template <class SC, int GM = G_DEFAULT>
hipError_t by_type(int S, bool f64, const BMember1* mem, int count, hipStream_t stream) {
  constexpr bool GD = guard_of<double, SC::N, GM>(), GF = guard_of<float, SC::N, GM>();
  if (f64) {
    if (S == 1) return launch<double, SC, 1, GD>(mem, count, stream);
    if (S == 2) return launch<double, SC, 2, GD>(mem, count, stream);
  } else {
    if (S == 1) return launch<float, SC, 1, GF>(mem, count, stream);
    if (S == 2) return launch<float, SC, 2, GF>(mem, count, stream);
  }
  return hipErrorInvalidValue;
}

// variants of one tuned length N <= 4096: 0 the default E8 schedule, 1 the
// same with the other twiddle policy, 2 E4 and 3 E16 (recomputed twiddles);
// N = 8192: 0 E8, 1 E16 (both recomputed).  Two surfaces of 1024 points: 0
// the four-wave body (the single-plan kernel there), 4 the default E8.
template <int N, class DEF>
hipError_t tuned(int variant, int S, bool f64, const BMember1* mem, int count,
                 hipStream_t stream) {
  if constexpr (N == w4::N) {
    if (S == 2 && variant == 0) return launch_w4(f64, mem, count, stream);
    if (S == 2 && variant == 4) return by_type<DEF, G_DEFAULT>(S, f64, mem, count, stream);
  }
  if (variant == 0) return by_type<DEF, G_DEFAULT>(S, f64, mem, count, stream);
  if constexpr (N <= 4096) {
    if (variant == 1) return by_type<DEF, G_OTHER>(S, f64, mem, count, stream);
    if (variant == 2) return by_type<typename Alt<N>::E4, G_ON>(S, f64, mem, count, stream);
    if (variant == 3) return by_type<typename Alt<N>::E16, G_ON>(S, f64, mem, count, stream);
  } else {
    if (variant == 1) return by_type<typename Alt<N>::E16, G_ON>(S, f64, mem, count, stream);
  }
  return hipErrorInvalidValue;
}

}  // namespace

int k1b_variants(int n, int S) {
  if (n == w4::N && S == 2) return 5;
  switch (n) {
    case 512: case 1024: case 2048: case 4096: return 4;
    case 8192: return 2;
    case 16: case 32: case 64: case 128: case 256: return 1;
    default: return 0;
  }
}

const char* k1b_variant_name(int n, int S, int variant, bool f64) {
  const bool g = f64 ? guard_default<double>(n) : guard_default<float>(n);
  if (n == w4::N && S == 2) {
    if (variant == 0) return "four waves, radix 8.8.4.4 (four-step), wave-local exchanges";
    if (variant == 4) variant = 0;
  }
  if (variant == 0 || (variant == 1 && n <= 4096)) {
    const bool guarded = (variant == 0) ? g : !g;
    switch (n) {
      case 16: return "E4 radix 4.4";
      case 32: return "E8 radix 8.4";
      case 64: return "E8 radix 8.8";
      case 128: return "E8 radix 8.4.4";
      case 256: return "E8 radix 8.8.4";
      case 512: return guarded ? "E8 radix 8.8.8, recomputed twiddles" : "E8 radix 8.8.8";
      case 1024: return guarded ? "E8 radix 8.4.4.8, recomputed twiddles" : "E8 radix 8.4.4.8";
      case 2048: return guarded ? "E8 radix 8.8.4.8, recomputed twiddles" : "E8 radix 8.8.4.8";
      case 4096: return guarded ? "E8 radix 8.8.8.8, recomputed twiddles" : "E8 radix 8.8.8.8";
      case 8192: return "E8 radix 8.8.8.8.2, recomputed twiddles";
      default: return "?";
    }
  }
  if (n == 8192) return variant == 1 ? "E16 radix 8.8.8.16, recomputed twiddles" : "?";
  if (variant == 2) {
    switch (n) {
      case 512: return "E4 radix 4.4.4.4.2, recomputed twiddles";
      case 1024: return "E4 radix 4.4.4.4.4, recomputed twiddles";
      case 2048: return "E4 radix 4.4.4.4.4.2, recomputed twiddles";
      case 4096: return "E4 radix 4.4.4.4.4.4, recomputed twiddles";
      default: return "?";
    }
  }
  if (variant == 3) {
    switch (n) {
      case 512: return "E16 radix 16.8.4, recomputed twiddles";
      case 1024: return "E16 radix 16.16.4, recomputed twiddles";
      case 2048: return "E16 radix 16.16.8, recomputed twiddles";
      case 4096: return "E16 radix 16.16.16, recomputed twiddles";
      default: return "?";
    }
  }
  return "?";
}

hipError_t k1b_launch(int n, int S, bool f64, int variant, const BMember1* mem, int count,
                      hipStream_t stream) {
  if (count <= 0) return hipSuccess;
  if (variant < 0 || variant >= k1b_variants(n, S)) return hipErrorInvalidValue;
  using namespace s1d;
  switch (n) {
    case 16: return by_type<S16>(S, f64, mem, count, stream);
    case 32: return by_type<S32>(S, f64, mem, count, stream);
    case 64: return by_type<S64>(S, f64, mem, count, stream);
    case 128: return by_type<S128>(S, f64, mem, count, stream);
    case 256: return by_type<S256>(S, f64, mem, count, stream);
    case 512: return tuned<512, S512>(variant, S, f64, mem, count, stream);
    case 1024: return tuned<1024, S1024>(variant, S, f64, mem, count, stream);
    case 2048: return tuned<2048, S2048>(variant, S, f64, mem, count, stream);
    case 4096: return tuned<4096, S4096>(variant, S, f64, mem, count, stream);
    case 8192: return tuned<8192, S8192>(variant, S, f64, mem, count, stream);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace sop
