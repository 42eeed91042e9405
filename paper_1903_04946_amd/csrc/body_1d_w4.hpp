// body_1d_w4.hpp -- the composed time step of a two-surface 1024-point
// wavepacket on four waves, one per SIMD of the compute unit.
//
// Same step as run_1d (Sec. "Dynamic Fourier method"; the pruned action
// sequence of Sec. "Pruning splitting coefficients"), with the work laid out
// so that all four SIMDs issue FP64 arithmetic and two of the three
// exchanges of a transform stay inside one wave:
//
// * 256 threads hold 8 values each; lane bit 5 selects the surface, so a
//   lane transforms one surface's values and lanes l and l + 32 hold the two
//   surfaces at the same points.
// * The DFT of length 1024 is the mixed-radix Cooley-Tukey factorisation
//   8 x 8 x 4 x 4 written as nested four-step transforms:
//       x = 128 x1 + 16 y1 + 4 z1 + z2,   k = k1 + 8 k1' + 64 k1'' + 256 k2'',
//   radix-8 DFT over x1, twiddle w_1024^(x2 k1) (x2 = x mod 128), radix-8
//   over y1, twiddle w_128^(y2 k1') (y2 = x mod 16), radix-4 over z1, twiddle
//   w_16^(z2 k1''), radix-4 over z2.  The inverse runs the same steps in
//   reverse order with conjugate roots (the unnormalised inverse DFT; the
//   1/N sits in the kinetic factors).
// * Ownership (wave w, lane l = 32 s + a, register r):
//       position side   x = 128 r + 4 a + w
//       after stage 1   lane (y1, z1) = (a / 4, a % 4), register k1
//       after stage 2   lane (k1, z1), register k1'
//       after stage 3   lane (k1, c), register (k1'' = r % 4, c2 = r / 4),
//                       where k1' = c + 4 c2; wave z2
//       frequency side  k = a / 4 + 8 (a % 4 + 4 (r / 4)) + 64 w + 256 (r % 4)
// * Exchanges A (stage 1 -> 2) and B (2 -> 3) permute register and lane
//   bits inside a wave through that wave's own LDS region.  A wavefront's LDS
//   operations complete in issue order, so they need only a compiler fence,
//   no workgroup barrier.  Exchange C (3 -> 4) permutes register and wave
//   bits through a shared region behind one barrier.  The inverse transform's
//   exchange C writes exactly the slots the same thread read in the forward
//   one and reads the slots it wrote there, so the one buffer needs no
//   second barrier: a thread only ever overwrites slots it has already read.
// * The potential action pairs the two surfaces of a point in one lane by
//   exchanging register halves between lanes l and l + 32 (v_permlane32_swap),
//   applies the S x S matvec to four points per lane, and swaps back.
#pragma once

#include "fft_core.hpp"
#include "internal.hpp"

namespace sop {
namespace w4 {

constexpr int N = 1024;
constexpr int kThreads = 256;
constexpr int kRow = 36;               // slots per k1 row of a wave region (32 + 4 padding)
constexpr int kSurf = 8 * kRow;        // slots per surface of a wave region
constexpr int kWave = 2 * kSurf;       // slots per wave region
constexpr int kCross = 4 * kWave;      // first slot of the shared region
constexpr int kSlots = kCross + 2 * N;  // LDS slots of one workgroup
template <typename T>
constexpr size_t lds_bytes() {
  return (size_t)kSlots * sizeof(cx<T>);
}

// Compiler fence for LDS traffic within one wave (the hardware already keeps
// a wave's LDS operations in order).
__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront", "local");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront", "local");
}
// Workgroup barrier ordering LDS only: global loads in flight (the kinetic
// factors) stay in flight across it.
__device__ __forceinline__ void lds_barrier() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
  __builtin_amdgcn_s_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}
// LDS slot of register r in each exchange, on its position side (_t) and its
// frequency side (_f).  The padding of the wave rows (36 slots for 32) and the
// XOR in exchange B keep every 8-lane group of a 16-byte access on distinct
// banks.
struct Map {
  int wa;  // wave region of this lane's surface
  int a, w, l;
  __device__ __forceinline__ Map(int tid) {
    l = tid & 63;
    w = tid >> 6;
    a = l & 31;
    wa = w * kWave + (l >> 5) * kSurf;
  }
  // A: element (k1, y1, z1) at row k1, column 4 y1 + z1
  __device__ __forceinline__ int a_t(int r) const { return wa + r * kRow + a; }
  __device__ __forceinline__ int a_f(int r) const { return wa + (a >> 2) * kRow + 4 * r + (a & 3); }
  // B: element (k1, k1' = c + 4 c2, z1) at row k1, column 16 c2 + 4 z1 + (c xor z1)
  __device__ __forceinline__ int b_t(int r) const {
    return wa + (a >> 2) * kRow + (r >> 2) * 16 + (a & 3) * 4 + ((r & 3) ^ (a & 3));
  }
  __device__ __forceinline__ int b_f(int r) const {
    return wa + (a >> 2) * kRow + (r >> 2) * 16 + (r & 3) * 4 + ((a & 3) ^ (r & 3));
  }
  // C: element (k1'', z2, c2, lane) of the shared region
  __device__ __forceinline__ int c_t(int r) const {
    return kCross + (((r & 3) * 4 + w) * 2 + (r >> 2)) * 64 + l;
  }
  __device__ __forceinline__ int c_f(int r) const {
    return kCross + ((w * 4 + (r & 3)) * 2 + (r >> 2)) * 64 + l;
  }
};

// Exchange inside the wave: write through `wr`, read through `rd`.
template <typename T, class WR, class RD>
__device__ __forceinline__ void xwave(cx<T> (&v)[8], cx<T>* lds, WR wr, RD rd) {
#pragma unroll
  for (int r = 0; r < 8; ++r) lds[wr(r)] = v[r];
  wave_sync();
#pragma unroll
  for (int r = 0; r < 8; ++r) v[r] = lds[rd(r)];
  wave_sync();
}
// Exchange across the waves (one barrier; see the header for the second).
template <typename T, class WR, class RD>
__device__ __forceinline__ void xcross(cx<T> (&v)[8], cx<T>* lds, WR wr, RD rd) {
#pragma unroll
  for (int r = 0; r < 8; ++r) lds[wr(r)] = v[r];
  lds_barrier();
#pragma unroll
  for (int r = 0; r < 8; ++r) v[r] = lds[rd(r)];
  wave_sync();
}

// a * F, or a * conj(F) when C
template <bool C, typename T>
__device__ __forceinline__ cx<T> fmul_c(cx<T> a, const Fac<T>& F) {
  if constexpr (!C) {
    return fmul(a, F);
  } else {
    Fac<T> G = F;
    G.w.im = -G.w.im;
    if constexpr (std::is_same<T, float>::value) G.lo.im = -G.lo.im;
    return fmul(a, G);
  }
}

// Twiddles of the three inner steps, fixed per thread for the whole run.
template <typename T>
struct Tw {
  Fac<T> t1[7], t2[7], t3[3];
  __device__ __forceinline__ void load(const cx<T>* __restrict__ tw, const Map& m) {
    const int x2 = 4 * m.a + m.w;            // x mod 128 on the position side
    const int y2 = 4 * (m.a & 3) + m.w;      // x mod 16 after stage 1
#pragma unroll
    for (int j = 1; j < 8; ++j) {
      t1[j - 1] = load_fac(tw, x2 * j, (T)1);        // w_1024^(x2 k1)
      t2[j - 1] = load_fac(tw, 8 * y2 * j, (T)1);    // w_128^(y2 k1')
    }
#pragma unroll
    for (int j = 1; j < 4; ++j) t3[j - 1] = load_fac(tw, 64 * m.w * j, (T)1);  // w_16^(z2 k1'')
  }
};

template <typename T>
__device__ __forceinline__ void forward(cx<T> (&v)[8], cx<T>* lds, const Map& m, const Tw<T>& tw) {
  dft<8, false>(v);
#pragma unroll
  for (int r = 1; r < 8; ++r) v[r] = fmul(v[r], tw.t1[r - 1]);
  xwave(v, lds, [&](int r) { return m.a_t(r); }, [&](int r) { return m.a_f(r); });
  dft<8, false>(v);
#pragma unroll
  for (int r = 1; r < 8; ++r) v[r] = fmul(v[r], tw.t2[r - 1]);
  xwave(v, lds, [&](int r) { return m.b_t(r); }, [&](int r) { return m.b_f(r); });
  dft<4, false>(v);
  dft<4, false>(v + 4);
#pragma unroll
  for (int r = 1; r < 8; ++r)
    if (r & 3) v[r] = fmul(v[r], tw.t3[(r & 3) - 1]);
  xcross(v, lds, [&](int r) { return m.c_t(r); }, [&](int r) { return m.c_f(r); });
  dft<4, false>(v);
  dft<4, false>(v + 4);
}

template <typename T>
__device__ __forceinline__ void inverse(cx<T> (&v)[8], cx<T>* lds, const Map& m, const Tw<T>& tw) {
  dft<4, true>(v);
  dft<4, true>(v + 4);
  xcross(v, lds, [&](int r) { return m.c_f(r); }, [&](int r) { return m.c_t(r); });
#pragma unroll
  for (int r = 1; r < 8; ++r)
    if (r & 3) v[r] = fmul_c<true>(v[r], tw.t3[(r & 3) - 1]);
  dft<4, true>(v);
  dft<4, true>(v + 4);
  xwave(v, lds, [&](int r) { return m.b_f(r); }, [&](int r) { return m.b_t(r); });
#pragma unroll
  for (int r = 1; r < 8; ++r) v[r] = fmul_c<true>(v[r], tw.t2[r - 1]);
  dft<8, true>(v);
  xwave(v, lds, [&](int r) { return m.a_f(r); }, [&](int r) { return m.a_t(r); });
#pragma unroll
  for (int r = 1; r < 8; ++r) v[r] = fmul_c<true>(v[r], tw.t1[r - 1]);
  dft<8, true>(v);
}

// Exchanges lanes 32-63 of `hi` with lanes 0-31 of `lo`.
template <typename T>
__device__ __forceinline__ void swap_halves(cx<T>& hi, cx<T>& lo) {
  constexpr int W = (int)(sizeof(cx<T>) / 4);
  struct Words {
    uint32_t u[W];
  };
  Words h = __builtin_bit_cast(Words, hi), o = __builtin_bit_cast(Words, lo);
#pragma unroll
  for (int i = 0; i < W; ++i) {
    const auto p = __builtin_amdgcn_permlane32_swap(h.u[i], o.u[i], false, false);
    h.u[i] = p[0];
    o.u[i] = p[1];
  }
  hi = __builtin_bit_cast(cx<T>, h);
  lo = __builtin_bit_cast(cx<T>, o);
}

}  // namespace w4

// The step loop on a state held in registers.  CONJ applies conj(U) and
// conj(F), which is U(-dt): a compile-time flag, so that the sign folds into
// the products where a factor is used and does not pull its load forward.
template <typename T, bool CONJ>
__device__ __forceinline__ void steps_w4(cx<T> (&v)[8], const w4::Map& m, const w4::Tw<T>& tws,
                                         const cx<T>* __restrict__ vexp,
                                         const cx<T>* __restrict__ kin,
                                         const int* __restrict__ prog, int nact, int64_t nsteps,
                                         cx<T>* lds) {
  using namespace w4;
  const int s = m.l >> 5;
  for (int64_t step = 0; step < nsteps; ++step) {
    for (int a = 0; a < nact; ++a) {
      const int code = prog[a];
      const int idx = code & 0xffff;
      if ((code >> 16) == OP_V) {
        const cx<T>* U = vexp + (size_t)idx * 3 * N * Split<T>::rep;
        Fac<T> u[4][3];
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          const int x = 128 * (i + 4 * s) + 4 * m.a + m.w;
#pragma unroll
          for (int e = 0; e < 3; ++e) {
            u[i][e] = load_fac(U, e * N + x, (T)1);
            if constexpr (CONJ) {
              u[i][e].w.im = -u[i][e].w.im;
              if constexpr (std::is_same<T, float>::value) u[i][e].lo.im = -u[i][e].lo.im;
            }
          }
        }
        // lanes 0-31 receive surface 1 of registers 0-3, lanes 32-63 surface 0
        // of registers 4-7: (v[i], v[4 + i]) is then the pair at x(i + 4 s)
#pragma unroll
        for (int i = 0; i < 4; ++i) swap_halves(v[i], v[4 + i]);
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          cx<T> p[2] = {v[i], v[4 + i]};
          apply_u_fac<T, 2>(p, u[i]);
          v[i] = p[0];
          v[4 + i] = p[1];
        }
#pragma unroll
        for (int i = 0; i < 4; ++i) swap_halves(v[i], v[4 + i]);
      } else {
        // the factors are requested before the forward transform, which
        // hides their latency (requesting the next potential action's
        // entries here as well measured slower: the registers they hold
        // make the compiler serialise the loads)
        const cx<T>* F = kin + (size_t)idx * N * Split<T>::rep;
        Fac<T> kf[8];
#pragma unroll
        for (int r = 0; r < 8; ++r)
          kf[r] = load_fac(F, (m.a >> 2) + 8 * ((m.a & 3) + 4 * (r >> 2)) + 64 * m.w + 256 * (r & 3),
                           (T)1);
        forward(v, lds, m, tws);
#pragma unroll
        for (int r = 0; r < 8; ++r) v[r] = fmul_c<CONJ>(v[r], kf[r]);
        inverse(v, lds, m, tws);
      }
    }
  }
}

// The composed step (arguments as in run_1d, S = 2, N = 1024, 256 threads,
// w4::lds_bytes<T>() bytes of LDS).
template <typename T>
__device__ __forceinline__ void run_1d_w4(cx<T>* __restrict__ psi, const cx<T>* __restrict__ vexp,
                                          const cx<T>* __restrict__ kin,
                                          const cx<T>* __restrict__ tw,
                                          const int* __restrict__ prog, int nact, int64_t nsteps,
                                          int conj, cx<T>* lds) {
  using namespace w4;
  const w4::Map m((int)threadIdx.x);
  const int s = m.l >> 5;
  Tw<T> tws;
  tws.load(tw, m);
  cx<T> v[8];
#pragma unroll
  for (int r = 0; r < 8; ++r) {
    v[r] = psi[s * N + 128 * r + 4 * m.a + m.w];
    // consumed here, so no load of psi is outstanding inside the step loop
    asm volatile("" : "+v"(v[r].re), "+v"(v[r].im));
  }
  if (conj)
    steps_w4<T, true>(v, m, tws, vexp, kin, prog, nact, nsteps, lds);
  else
    steps_w4<T, false>(v, m, tws, vexp, kin, prog, nact, nsteps, lds);
#pragma unroll
  for (int r = 0; r < 8; ++r) psi[s * N + 128 * r + 4 * m.a + m.w] = v[r];
}

}  // namespace sop
