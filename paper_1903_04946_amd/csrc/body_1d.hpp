// body_1d.hpp -- the composed time step of a one-dimensional wavepacket as a
// device function run by one workgroup.
//
// The S-surface state stays in registers (radix-R_first ownership) for all
// nsteps x (N_A + N_B) actions of the pruned sequence (Sec. "Pruning
// splitting coefficients"); only the FFT stage exchanges touch LDS, and HBM
// sees psi at entry and exit.  A potential action is the S x S matvec with
// the stored table exp(-i a dt V(x)/hbar) of its unique coefficient
// (Eq. range_index_unq); a kinetic action is forward FFT -> phase (with 1/N
// folded in) -> inverse FFT (Sec. "Dynamic Fourier method").  conj = 1
// conjugates every table, which is U(-dt).
#pragma once

#include "fft_core.hpp"
#include "internal.hpp"

namespace sop {

namespace s1d {
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
}  // namespace s1d

// LDS slots of one pencil: one padding slot per 16 elements.
template <class SC>
constexpr int lds_pencil() {
  return SC::N + SC::N / 16;
}

// GUARD: pass the thread index through opaque() for every transform and
// action, so that twiddles and addresses are recomputed instead of being
// held for the whole run.  Measured per step on gfx950 (two surfaces, FP64):
// N = 8192 55 us guarded vs 141 us held (spilled); 512 and 2048 slightly
// faster guarded; 1024 slightly faster without.  At N = 4096 the held FP64
// kernel spills (256 VGPRs and 400 bytes of scratch a lane) and the guarded
// one does not (178 VGPRs): 17.8 against 20.8 us a substep; in FP32 nothing
// spills and holding is faster (12.3 against 14.5 us).
template <typename T>
constexpr bool guard_default(int n) {
  return n == 512 || n == 2048 || n >= 8192 || (n == 4096 && sizeof(T) == 8);
}
template <bool GUARD>
__device__ __forceinline__ int guard(int t) {
  if constexpr (GUARD) return opaque(t);
  else return t;
}

// PL = pencils exchanged through LDS at once (S, or 1 when S pencils do not
// fit).  `lds` holds PL padded pencils.  With one pencil of buffer and two
// surfaces the two transforms run interleaved (fft_forward_pair).
template <typename T, class SC, int S, int PL, bool GUARD = guard_default<T>(SC::N)>
__device__ __forceinline__ void run_1d(cx<T>* __restrict__ psi, const cx<T>* __restrict__ vexp,
                                       const cx<T>* __restrict__ kin,
                                       const cx<T>* __restrict__ tw,
                                       const int* __restrict__ prog, int nact, int64_t nsteps,
                                       int conj, cx<T>* lds) {
  const int t0 = threadIdx.x;
  constexpr int N = SC::N, E = SC::E, NE = S * (S + 1) / 2;
  const T csign = conj ? (T)-1 : (T)1;
  cx<T> v[S][E];
#pragma unroll
  for (int s = 0; s < S; ++s)
#pragma unroll
    for (int q = 0; q < E; ++q) v[s][q] = psi[s * N + own_idx<N, E, SC::RF>(t0, q)];
  const LayPadded lay{0, lds_pencil<SC>()};

  for (int64_t step = 0; step < nsteps; ++step) {
    for (int a = 0; a < nact; ++a) {
      const int code = prog[a];
      const int idx = code & 0xffff;
      const int t = guard<GUARD>(t0);
      if ((code >> 16) == OP_V) {
        // table entries are (rounded, residue) pairs in FP32
        const cx<T>* U = vexp + (size_t)idx * NE * N * Split<T>::rep;
#pragma unroll
        for (int q = 0; q < E; ++q) {
          const int x = own_idx<N, E, SC::RF>(t, q);
          Fac<T> u[NE];
#pragma unroll
          for (int e = 0; e < NE; ++e) u[e] = load_fac(U, e * N + x, csign);
          cx<T> w[S];
#pragma unroll
          for (int s = 0; s < S; ++s) w[s] = v[s][q];
          apply_u_fac<T, S>(w, u);
#pragma unroll
          for (int s = 0; s < S; ++s) v[s][q] = w[s];
        }
      } else {
        if constexpr (PL == S && S == 2) {
          fft_forward_pair2<SC>(v, lds, lay, tw, guard<GUARD>(t0));
        } else if constexpr (PL == S) {
          fft_forward<SC, S>(v, lds, lay, tw, guard<GUARD>(t0));
        } else if constexpr (S == 2) {
          fft_forward_pair<SC>(v, lds, lay, tw, guard<GUARD>(t0));
        } else {
#pragma unroll
          for (int s = 0; s < S; ++s) fft_forward<SC, 1>(v + s, lds, lay, tw, guard<GUARD>(t0));
        }
        const cx<T>* F = kin + (size_t)idx * N * Split<T>::rep;
#pragma unroll
        for (int q = 0; q < E; ++q) {
          const Fac<T> f = load_fac(F, own_idx<N, E, SC::RL>(t, q), csign);
#pragma unroll
          for (int s = 0; s < S; ++s) v[s][q] = fmul(v[s][q], f);
        }
        if constexpr (PL == S && S == 2) {
          fft_inverse_pair2<SC>(v, lds, lay, tw, guard<GUARD>(t0));
        } else if constexpr (PL == S) {
          fft_inverse<SC, S>(v, lds, lay, tw, guard<GUARD>(t0));
        } else if constexpr (S == 2) {
          fft_inverse_pair<SC>(v, lds, lay, tw, guard<GUARD>(t0));
        } else {
#pragma unroll
          for (int s = 0; s < S; ++s) fft_inverse<SC, 1>(v + s, lds, lay, tw, guard<GUARD>(t0));
        }
      }
    }
  }
#pragma unroll
  for (int s = 0; s < S; ++s)
#pragma unroll
    for (int q = 0; q < E; ++q) psi[s * N + own_idx<N, E, SC::RF>(t0, q)] = v[s][q];
}

}  // namespace sop
