// fft_core.hpp -- register/LDS Stockham FFT building blocks for gfx950.
//
// A pencil of length N is held by N/E threads, E complex values each.  A
// stage of radix R with sub-transform length L (product of the earlier
// radices) lets thread t own the butterflies j = t + (N/E) b, b < E/R; the
// inputs of butterfly j are the elements j + m N/R (m < R), its twiddles are
// exp(-+2 pi i k m/(L R)) with k = j mod L, and its outputs land at
// (j - k) R + k + m L (Stockham auto-sort: natural order in and out, no bit
// reversal).  Between stages the values go through LDS; after the last
// stage thread t owns exactly the elements of a radix-R_last first stage, so
// a forward transform (radices R_1..R_k) followed by an inverse one with the
// radices reversed (R_k..R_1) needs no exchange at the turn, and pointwise
// work (the kinetic phase, the potential matvec) happens in registers.
//
// The transforms are the unnormalised DFTs of the dynamic Fourier method
// (Sec. "Dynamic Fourier method"): forward exp(-2 pi i jk/N), inverse
// exp(+2 pi i jk/N); the 1/N of the inverse is folded into the kinetic
// factors by the planner.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <type_traits>

namespace sop {

template <typename T>
struct __align__(2 * sizeof(T)) cx {
  T re, im;
};

template <typename T>
__device__ __forceinline__ cx<T> cadd(cx<T> a, cx<T> b) { return {a.re + b.re, a.im + b.im}; }
template <typename T>
__device__ __forceinline__ cx<T> csub(cx<T> a, cx<T> b) { return {a.re - b.re, a.im - b.im}; }
template <typename T>
__device__ __forceinline__ cx<T> cmul(cx<T> a, cx<T> b) {
  return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re};
}
template <typename T>
__device__ __forceinline__ cx<T> cconj(cx<T> a) { return {a.re, -a.im}; }
// multiply by -i (forward) or +i (inverse)
template <bool INV, typename T>
__device__ __forceinline__ cx<T> mul_mi(cx<T> a) {
  if (INV) return {-a.im, a.re};
  return {a.im, -a.re};
}

// ----------------------------------------------------------------- FP32 products
// In FP32 every fixed unit-modulus factor -- a twiddle, a radix constant such
// as cos(pi/4), a kinetic factor -- rounds to a value whose modulus is off 1
// by the same amount at every application.  Within one transform that is
// harmless, but the time step applies the same factors thousands of times,
// and the deterministic bias compounds into a norm drift linear in the number
// of substeps (about 1e-7 a substep at 32^3, mostly loss: the rounded twiddles
// of small transforms all lie inside the unit circle), far above the
// random-walk growth of ordinary roundings.  FP32 products with such factors
// therefore carry the rounding residue lo = value - rounded: x (w + lo) is
// formed with fused multiply-adds, so the only roundings are those of the
// sums, which have no preferred sign.  FP32 plans store every twiddle and
// kinetic factor as the pair (rounded, residue), 16 bytes read by one load:
// a block of n factors holds Split<float>::rep * n complex values.
template <typename T>
struct Split {
  static constexpr int rep = 1;
};
template <>
struct Split<float> {
  static constexpr int rep = 2;
};

// A factor read from a (split) table, conjugated when csign = -1.
template <typename T>
struct Fac {
  cx<T> w;
};
template <>
struct Fac<float> {
  cx<float> w, lo;
};
typedef float sop_f32x4 __attribute__((ext_vector_type(4)));
// Entry i of a factor block.
template <typename T>
__device__ __forceinline__ Fac<T> load_fac(const cx<T>* __restrict__ f, int i, T csign) {
  Fac<T> F;
  if constexpr (std::is_same<T, float>::value) {
    const sop_f32x4 q = *reinterpret_cast<const sop_f32x4*>(f + 2 * i);
    F.w = {q.x, csign * q.y};
    F.lo = {q.z, csign * q.w};
  } else {
    F.w = f[i];
    F.w.im *= csign;
  }
  return F;
}
// a (w + lo): the residue terms enter below the rounded products.
__device__ __forceinline__ cx<float> cmul_lo(cx<float> a, cx<float> w, cx<float> lo) {
  const float cr = __builtin_fmaf(a.re, lo.re, -a.im * lo.im);
  const float ci = __builtin_fmaf(a.re, lo.im, a.im * lo.re);
  return {__builtin_fmaf(a.re, w.re, __builtin_fmaf(-a.im, w.im, cr)),
          __builtin_fmaf(a.re, w.im, __builtin_fmaf(a.im, w.re, ci))};
}
template <typename T>
__device__ __forceinline__ cx<T> fmul(cx<T> a, const Fac<T>& F) {
  if constexpr (std::is_same<T, float>::value) return cmul_lo(a, F.w, F.lo);
  else return cmul(a, F.w);
}

// ----------------------------------------------------------------- radix DFTs
// Radix constants; in FP32 with their rounding residues (K<float>::*_lo).
template <typename T>
struct K {
  static constexpr T r2 = (T)0.70710678118654752440084436210484903928;   // cos(pi/4)
  static constexpr T c8 = (T)0.92387953251128675612818318939678828682;   // cos(pi/8)
  static constexpr T s8 = (T)0.38268343236508977172845998403039886676;   // sin(pi/8)
  static constexpr T s3 = (T)0.86602540378443864676372317075293618347;   // sin(pi/3)
};
template <>
struct K<float> {
  static constexpr double R2 = 0.70710678118654752440084436210484903928;
  static constexpr double C8 = 0.92387953251128675612818318939678828682;
  static constexpr double S8 = 0.38268343236508977172845998403039886676;
  static constexpr double S3 = 0.86602540378443864676372317075293618347;
  static constexpr float r2 = (float)R2, r2_lo = (float)(R2 - (double)r2);
  static constexpr float c8 = (float)C8, c8_lo = (float)(C8 - (double)c8);
  static constexpr float s8 = (float)S8, s8_lo = (float)(S8 - (double)s8);
  static constexpr float s3 = (float)S3, s3_lo = (float)(S3 - (double)s3);
};
template <typename T> __device__ __forceinline__ constexpr T lo_r2() {
  if constexpr (std::is_same<T, float>::value) return K<float>::r2_lo; else return (T)0;
}
template <typename T> __device__ __forceinline__ constexpr T lo_c8() {
  if constexpr (std::is_same<T, float>::value) return K<float>::c8_lo; else return (T)0;
}
template <typename T> __device__ __forceinline__ constexpr T lo_s8() {
  if constexpr (std::is_same<T, float>::value) return K<float>::s8_lo; else return (T)0;
}
template <typename T> __device__ __forceinline__ constexpr T lo_s3() {
  if constexpr (std::is_same<T, float>::value) return K<float>::s3_lo; else return (T)0;
}
// x * constant (hi + lo in FP32)
template <typename T>
__device__ __forceinline__ T mulk(T x, T hi, T lo) {
  if constexpr (std::is_same<T, float>::value) return __builtin_fmaf(x, hi, x * lo);
  else return x * hi;
}

template <bool INV, typename T>
__device__ __forceinline__ void dft2(cx<T>* v) {
  cx<T> a = v[0], b = v[1];
  v[0] = cadd(a, b);
  v[1] = csub(a, b);
}

template <bool INV, typename T>
__device__ __forceinline__ void dft3(cx<T>* v) {
  // y0 = x0 + x1 + x2; y1,2 = x0 - (x1+x2)/2 -+ i sin(pi/3) (x1 - x2) (forward)
  cx<T> s = cadd(v[1], v[2]);
  cx<T> d = csub(v[1], v[2]);
  cx<T> h = {v[0].re - (T)0.5 * s.re, v[0].im - (T)0.5 * s.im};
  const T k3 = K<T>::s3, k3l = lo_s3<T>();
  cx<T> e = mul_mi<INV>(cx<T>{mulk(d.re, k3, k3l), mulk(d.im, k3, k3l)});
  v[0] = cadd(v[0], s);
  v[1] = cadd(h, e);
  v[2] = csub(h, e);
}

template <bool INV, typename T>
__device__ __forceinline__ void dft4(cx<T>* v) {
  cx<T> a = cadd(v[0], v[2]), b = csub(v[0], v[2]);
  cx<T> c = cadd(v[1], v[3]), d = mul_mi<INV>(csub(v[1], v[3]));
  v[0] = cadd(a, c);
  v[2] = csub(a, c);
  v[1] = cadd(b, d);
  v[3] = csub(b, d);
}

// x * exp(-+ i pi/4)
template <bool INV, typename T>
__device__ __forceinline__ cx<T> w8_1(cx<T> a) {
  const T r = K<T>::r2, rl = lo_r2<T>();
  if (INV) return {mulk(a.re - a.im, r, rl), mulk(a.re + a.im, r, rl)};
  return {mulk(a.re + a.im, r, rl), mulk(a.im - a.re, r, rl)};
}
// x * exp(-+ 3 i pi/4)
template <bool INV, typename T>
__device__ __forceinline__ cx<T> w8_3(cx<T> a) {
  const T r = K<T>::r2, rl = lo_r2<T>();
  if (INV) return {-mulk(a.re + a.im, r, rl), mulk(a.re - a.im, r, rl)};
  return {mulk(a.im - a.re, r, rl), -mulk(a.re + a.im, r, rl)};
}
// x * (c + i s) for a radix constant pair
template <typename T>
__device__ __forceinline__ cx<T> cmulk(cx<T> a, T c, T s, T cl, T sl) {
  if constexpr (std::is_same<T, float>::value) return cmul_lo(a, {c, s}, {cl, sl});
  else return cmul(a, cx<T>{c, s});
}

template <bool INV, typename T>
__device__ __forceinline__ void dft8(cx<T>* v) {
  cx<T> e[4] = {v[0], v[2], v[4], v[6]};
  cx<T> o[4] = {v[1], v[3], v[5], v[7]};
  dft4<INV>(e);
  dft4<INV>(o);
  o[1] = w8_1<INV>(o[1]);
  o[2] = mul_mi<INV>(o[2]);
  o[3] = w8_3<INV>(o[3]);
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    v[k] = cadd(e[k], o[k]);
    v[k + 4] = csub(e[k], o[k]);
  }
}

template <bool INV, typename T>
__device__ __forceinline__ void dft16(cx<T>* v) {
  cx<T> e[8], o[8];
#pragma unroll
  for (int k = 0; k < 8; ++k) {
    e[k] = v[2 * k];
    o[k] = v[2 * k + 1];
  }
  dft8<INV>(e);
  dft8<INV>(o);
  const T c = K<T>::c8, s = K<T>::s8, cl = lo_c8<T>(), sl = lo_s8<T>();
  const T sg = INV ? (T)1 : (T)-1;  // sign of the imaginary part of the twiddle
  // o[k] *= exp(sg * i * 2 pi k / 16), k = 1..7
  o[1] = cmulk(o[1], c, sg * s, cl, sg * sl);
  o[2] = w8_1<INV>(o[2]);
  o[3] = cmulk(o[3], s, sg * c, sl, sg * cl);
  o[4] = mul_mi<INV>(o[4]);
  o[5] = cmulk(o[5], -s, sg * c, -sl, sg * cl);
  o[6] = w8_3<INV>(o[6]);
  o[7] = cmulk(o[7], -c, sg * s, -cl, sg * sl);
#pragma unroll
  for (int k = 0; k < 8; ++k) {
    v[k] = cadd(e[k], o[k]);
    v[k + 8] = csub(e[k], o[k]);
  }
}

template <int R, bool INV, typename T>
__device__ __forceinline__ void dft(cx<T>* v) {
  if constexpr (R == 2) dft2<INV>(v);
  else if constexpr (R == 3) dft3<INV>(v);
  else if constexpr (R == 4) dft4<INV>(v);
  else if constexpr (R == 8) dft8<INV>(v);
  else if constexpr (R == 16) dft16<INV>(v);
  else static_assert(R == 2, "unsupported radix");
}

// ----------------------------------------------------------------- schedules
template <int... Rs>
struct RList {};

template <int R, int... Rs>
struct RHead {
  static constexpr int value = R;
};

// A pencil schedule: length N, E elements per thread, forward radices Fwd and
// inverse radices Inv = reverse(Fwd).
template <int N_, int E_, class Fwd_, class Inv_, int RF_, int RL_>
struct Sched {
  static constexpr int N = N_;
  static constexpr int E = E_;
  static constexpr int TPC = N_ / E_;  // threads per pencil
  static constexpr int RF = RF_;       // first forward radix (= last inverse radix)
  static constexpr int RL = RL_;       // last forward radix (= first inverse radix)
  using Fwd = Fwd_;
  using Inv = Inv_;
};

// Global accesses through buffer resources: the descriptor (base, extent)
// lives in SGPRs and every access takes one 32-bit VGPR offset, so all loads
// and stores of a thread share a handful of offset registers.  Accesses
// outside the extent read zero and drop writes instead of faulting.  The
// fourth descriptor word 0x00020000 is the raw 32-bit data format of the
// gfx9 family.
typedef unsigned int sop_u32x4 __attribute__((ext_vector_type(4)));
typedef unsigned int sop_u32x2 __attribute__((ext_vector_type(2)));

template <typename T>
__device__ __forceinline__ __amdgpu_buffer_rsrc_t rsrc(const cx<T>* p, uint32_t nelem) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<cx<T>*>(p), (short)0,
                                           (int)(nelem * (uint32_t)sizeof(cx<T>)), 0x00020000);
}
__device__ __forceinline__ cx<double> bld(__amdgpu_buffer_rsrc_t r, uint32_t idx, cx<double>*) {
  sop_u32x4 v = __builtin_amdgcn_raw_buffer_load_b128(r, (int)(idx * 16u), 0, 0);
  return __builtin_bit_cast(cx<double>, v);
}
__device__ __forceinline__ cx<float> bld(__amdgpu_buffer_rsrc_t r, uint32_t idx, cx<float>*) {
  sop_u32x2 v = __builtin_amdgcn_raw_buffer_load_b64(r, (int)(idx * 8u), 0, 0);
  return __builtin_bit_cast(cx<float>, v);
}
template <typename T>
__device__ __forceinline__ cx<T> ld(__amdgpu_buffer_rsrc_t r, uint32_t idx) {
  return bld(r, idx, (cx<T>*)nullptr);
}
// Entry idx of a factor table (Split<T>::rep complex values per entry: in
// FP32 the pair (rounded, residue), 16 bytes read by one load), conjugated
// when csign = -1.
template <typename T>
__device__ __forceinline__ Fac<T> ldfac(__amdgpu_buffer_rsrc_t r, uint32_t idx, T csign) {
  Fac<T> F;
  if constexpr (std::is_same<T, float>::value) {
    sop_u32x4 v = __builtin_amdgcn_raw_buffer_load_b128(r, (int)(idx * 16u), 0, 0);
    const sop_f32x4 q = __builtin_bit_cast(sop_f32x4, v);
    F.w = {q.x, csign * q.y};
    F.lo = {q.z, csign * q.w};
  } else {
    F.w = bld(r, idx, (cx<T>*)nullptr);
    F.w.im *= csign;
  }
  return F;
}
__device__ __forceinline__ void st(__amdgpu_buffer_rsrc_t r, uint32_t idx, cx<double> v) {
  __builtin_amdgcn_raw_buffer_store_b128(__builtin_bit_cast(sop_u32x4, v), r, (int)(idx * 16u), 0, 0);
}
__device__ __forceinline__ void st(__amdgpu_buffer_rsrc_t r, uint32_t idx, cx<float> v) {
  __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(sop_u32x2, v), r, (int)(idx * 8u), 0, 0);
}

// The thread index passed through an empty asm statement: the compiler can no
// longer prove two transforms use the same twiddle and LDS addresses, so it
// reloads each transform's twiddles instead of keeping those of every stage
// and surface live across the whole step (which spills large pencils).
__device__ __forceinline__ int opaque(int t) {
  asm volatile("" : "+v"(t));
  return t;
}

// Element index owned by thread t in register slot `slot` for a radix-R stage.
template <int N, int E, int R>
__device__ __forceinline__ int own_idx(int t, int slot) {
  const int b = slot / R, m = slot % R;
  return t + (N / E) * b + m * (N / R);
}

// ----------------------------------------------------------------- LDS layouts
// Pencil-fastest layout: offset = base + p * pstride + e * estride
struct LayStrided {
  int base, pstride, estride;
  __device__ __forceinline__ int off(int p, int e) const { return base + p * pstride + e * estride; }
};
// Element-fastest layout with one padding slot per 16 elements:
// offset = base + p * pstride + e + e/16
struct LayPadded {
  int base, pstride;
  __device__ __forceinline__ int off(int p, int e) const { return base + p * pstride + e + (e >> 4); }
};

// ----------------------------------------------------------------- stages
template <typename T, int N, int E, int R, int L, bool INV>
__device__ __forceinline__ void stage(cx<T> (&v)[E], int t, const cx<T>* __restrict__ tw) {
  constexpr int TPC = N / E;
#pragma unroll
  for (int b = 0; b < E / R; ++b) {
    if constexpr (L > 1) {
      const int j = t + TPC * b;
      const int k = j % L;
#pragma unroll
      for (int m = 1; m < R; ++m) {
        const Fac<T> w = load_fac(tw, (k * m) * (N / (L * R)), INV ? (T)-1 : (T)1);
        v[b * R + m] = fmul(v[b * R + m], w);
      }
    }
    dft<R, INV>(&v[b * R]);
  }
}

// Writes the outputs of a (R, L) stage to LDS and reads the inputs of the
// next stage (radix R2).  All P pencils of the thread go through together.
template <typename T, int N, int E, int R, int L, int R2, int P, class Lay>
__device__ __forceinline__ void exchange(cx<T> (*v)[E], cx<T>* lds, const Lay& lay, int t) {
  constexpr int TPC = N / E;
#pragma unroll
  for (int b = 0; b < E / R; ++b) {
    const int j = t + TPC * b;
    const int k = j % L;
    const int base = (j - k) * R + k;
#pragma unroll
    for (int p = 0; p < P; ++p)
#pragma unroll
      for (int m = 0; m < R; ++m) lds[lay.off(p, base + m * L)] = v[p][b * R + m];
  }
  __syncthreads();
#pragma unroll
  for (int b = 0; b < E / R2; ++b) {
    const int j = t + TPC * b;
#pragma unroll
    for (int p = 0; p < P; ++p)
#pragma unroll
      for (int m = 0; m < R2; ++m) v[p][b * R2 + m] = lds[lay.off(p, j + m * (N / R2))];
  }
  __syncthreads();
}

template <typename T, int N, int E, bool INV, int L, int P, class Lay, int R, int... Rest>
__device__ __forceinline__ void run_stages(cx<T> (*v)[E], cx<T>* lds, const Lay& lay,
                                           const cx<T>* __restrict__ tw, int t, RList<R, Rest...>) {
#pragma unroll
  for (int p = 0; p < P; ++p) stage<T, N, E, R, L, INV>(v[p], t, tw);
  if constexpr (sizeof...(Rest) > 0) {
    constexpr int R2 = RHead<Rest...>::value;
    exchange<T, N, E, R, L, R2, P>(v, lds, lay, t);
    run_stages<T, N, E, INV, L * R, P, Lay>(v, lds, lay, tw, t, RList<Rest...>{});
  }
}

// The two halves of exchange() for one pencil, in pencil slot p of the
// layout: the writes of a (R, L) stage's outputs, and the reads of the next
// stage's (radix R2) inputs.  The caller places the barriers.
template <typename T, int N, int E, int R, int L, int R2, class Lay>
__device__ __forceinline__ void exchange_write(const cx<T> (&v)[E], cx<T>* lds, const Lay& lay,
                                               int t, int p = 0) {
  constexpr int TPC = N / E;
#pragma unroll
  for (int b = 0; b < E / R; ++b) {
    const int j = t + TPC * b;
    const int k = j % L;
    const int base = (j - k) * R + k;
#pragma unroll
    for (int m = 0; m < R; ++m) lds[lay.off(p, base + m * L)] = v[b * R + m];
  }
}
template <typename T, int N, int E, int R2, class Lay>
__device__ __forceinline__ void exchange_read(cx<T> (&v)[E], const cx<T>* lds, const Lay& lay,
                                              int t, int p = 0) {
  constexpr int TPC = N / E;
#pragma unroll
  for (int b = 0; b < E / R2; ++b) {
    const int j = t + TPC * b;
#pragma unroll
    for (int m = 0; m < R2; ++m) v[b * R2 + m] = lds[lay.off(p, j + m * (N / R2))];
  }
}
// Two pencils through one single-pencil LDS buffer, the second half a stage
// behind the first: while one pencil's exchange reads are in flight, the
// other pencil's butterflies run, so that the arithmetic of one overlaps the
// LDS traffic of the other (the buffer holds one pencil, as when the two do
// not fit in LDS together; same stages, same arithmetic as two transforms in
// turn).  Precondition of each level: pencil 0 has done stage (R, L),
// pencil 1 has not.
template <typename T, int N, int E, bool INV, int L, class Lay, int R, int... Rest>
__device__ __forceinline__ void pair_levels(cx<T> (*v)[E], cx<T>* lds, const Lay& lay,
                                            const cx<T>* __restrict__ tw, int t,
                                            RList<R, Rest...>) {
  if constexpr (sizeof...(Rest) == 0) {
    stage<T, N, E, R, L, INV>(v[1], t, tw);
  } else {
    constexpr int R2 = RHead<Rest...>::value;
    exchange_write<T, N, E, R, L, R2>(v[0], lds, lay, t);
    __syncthreads();
    exchange_read<T, N, E, R2>(v[0], lds, lay, t);
    stage<T, N, E, R, L, INV>(v[1], t, tw);
    __syncthreads();
    exchange_write<T, N, E, R, L, R2>(v[1], lds, lay, t);
    __syncthreads();
    exchange_read<T, N, E, R2>(v[1], lds, lay, t);
    stage<T, N, E, R2, L * R, INV>(v[0], t, tw);
    __syncthreads();
    pair_levels<T, N, E, INV, L * R, Lay>(v, lds, lay, tw, t, RList<Rest...>{});
  }
}
// The same with a buffer for each pencil: two barriers a level, as when the
// two go through together, with each pencil's exchange reads in flight while
// the other pencil's butterflies run.
template <typename T, int N, int E, bool INV, int L, class Lay, int R, int... Rest>
__device__ __forceinline__ void pair2_levels(cx<T> (*v)[E], cx<T>* lds, const Lay& lay,
                                             const cx<T>* __restrict__ tw, int t,
                                             RList<R, Rest...>) {
  if constexpr (sizeof...(Rest) == 0) {
    stage<T, N, E, R, L, INV>(v[1], t, tw);
  } else {
    constexpr int R2 = RHead<Rest...>::value;
    exchange_write<T, N, E, R, L, R2>(v[0], lds, lay, t, 0);
    __syncthreads();
    exchange_read<T, N, E, R2>(v[0], lds, lay, t, 0);
    stage<T, N, E, R, L, INV>(v[1], t, tw);
    exchange_write<T, N, E, R, L, R2>(v[1], lds, lay, t, 1);
    __syncthreads();
    exchange_read<T, N, E, R2>(v[1], lds, lay, t, 1);
    stage<T, N, E, R2, L * R, INV>(v[0], t, tw);
    pair2_levels<T, N, E, INV, L * R, Lay>(v, lds, lay, tw, t, RList<Rest...>{});
  }
}
template <typename T, int N, int E, bool INV, class Lay, int R, int... Rest>
__device__ __forceinline__ void pair2_stages(cx<T> (*v)[E], cx<T>* lds, const Lay& lay,
                                             const cx<T>* __restrict__ tw, int t,
                                             RList<R, Rest...> rl) {
  stage<T, N, E, R, 1, INV>(v[0], t, tw);
  // no barrier at the end: the last reads of each buffer precede a barrier
  // that every thread passes before its next write to that buffer (the next
  // transform writes pencil 0's buffer first, pencil 1's after a barrier)
  pair2_levels<T, N, E, INV, 1, Lay>(v, lds, lay, tw, t, rl);
}
template <class SC, typename T, class Lay>
__device__ __forceinline__ void fft_forward_pair2(cx<T> (*v)[SC::E], cx<T>* lds, const Lay& lay,
                                                  const cx<T>* __restrict__ tw, int t) {
  pair2_stages<T, SC::N, SC::E, false, Lay>(v, lds, lay, tw, t, typename SC::Fwd{});
}
template <class SC, typename T, class Lay>
__device__ __forceinline__ void fft_inverse_pair2(cx<T> (*v)[SC::E], cx<T>* lds, const Lay& lay,
                                                  const cx<T>* __restrict__ tw, int t) {
  pair2_stages<T, SC::N, SC::E, true, Lay>(v, lds, lay, tw, t, typename SC::Inv{});
}

template <typename T, int N, int E, bool INV, class Lay, int R, int... Rest>
__device__ __forceinline__ void pair_stages(cx<T> (*v)[E], cx<T>* lds, const Lay& lay,
                                            const cx<T>* __restrict__ tw, int t,
                                            RList<R, Rest...> rl) {
  stage<T, N, E, R, 1, INV>(v[0], t, tw);
  pair_levels<T, N, E, INV, 1, Lay>(v, lds, lay, tw, t, rl);
}
// Forward / inverse transforms of the two pencils v[0], v[1] through a buffer
// of one pencil (orderings as fft_forward / fft_inverse).
template <class SC, typename T, class Lay>
__device__ __forceinline__ void fft_forward_pair(cx<T> (*v)[SC::E], cx<T>* lds, const Lay& lay,
                                                 const cx<T>* __restrict__ tw, int t) {
  pair_stages<T, SC::N, SC::E, false, Lay>(v, lds, lay, tw, t, typename SC::Fwd{});
}
template <class SC, typename T, class Lay>
__device__ __forceinline__ void fft_inverse_pair(cx<T> (*v)[SC::E], cx<T>* lds, const Lay& lay,
                                                 const cx<T>* __restrict__ tw, int t) {
  pair_stages<T, SC::N, SC::E, true, Lay>(v, lds, lay, tw, t, typename SC::Inv{});
}

// Forward transform of P pencils v[0..P-1]: input in radix-RF ownership,
// output in radix-RL ownership.
template <class SC, int P, typename T, class Lay>
__device__ __forceinline__ void fft_forward(cx<T> (*v)[SC::E], cx<T>* lds, const Lay& lay,
                                            const cx<T>* __restrict__ tw, int t) {
  run_stages<T, SC::N, SC::E, false, 1, P, Lay>(v, lds, lay, tw, t, typename SC::Fwd{});
}
// Inverse transform: input in radix-RL ownership, output in radix-RF ownership.
template <class SC, int P, typename T, class Lay>
__device__ __forceinline__ void fft_inverse(cx<T> (*v)[SC::E], cx<T>* lds, const Lay& lay,
                                            const cx<T>* __restrict__ tw, int t) {
  run_stages<T, SC::N, SC::E, true, 1, P, Lay>(v, lds, lay, tw, t, typename SC::Inv{});
}

// ----------------------------------------------------------------- phases
// Largest |x| that sincos_phase accepts (the quadrant count stays below 2^22,
// so its products with the 30-bit parts of pi/2 are exact).
constexpr double kPhaseMax = 1.0e6;

// sin x and cos x in FP64 for |x| <= kPhaseMax: Cody-Waite reduction
// x = k pi/2 + r with pi/2 = C1 + C2 + C3 (C1, C2 of 30 significant bits,
// together about 115 bits, computed from Machin's formula
// pi = 16 atan(1/5) - 4 atan(1/239)), then the Taylor series of sin and cos
// on |r| <= pi/4 through r^17 and r^18 (the first omitted terms are below
// 1e-19).  Short and branch-free, unlike the general library routine with its
// large-argument reduction.
__host__ __device__ __forceinline__ void sincos_phase(double x, double* sn, double* cs) {
  const double k = rint(x * 0.63661977236758138);  // 2/pi
  double r = fma(-k, 1.5707963276654482, x);      // C1 = 0x1.921fb548p+0
  r = fma(-k, -8.705515692000731e-10, r);         // C2 = -0x1.de973dc8p-31
  r = fma(-k, -3.50343439808993e-19, r);          // C3
  const double u = r * r;
  // sin r = r sum_{n<=8} (-u)^n / (2n+1)!, Horner from the top term
  double ps = 1.0 / 355687428096000.0;   // 1/17!
  ps = fma(ps, u, -1.0 / 1307674368000.0);  // 1/15!
  ps = fma(ps, u, 1.0 / 6227020800.0);      // 1/13!
  ps = fma(ps, u, -1.0 / 39916800.0);       // 1/11!
  ps = fma(ps, u, 1.0 / 362880.0);          // 1/9!
  ps = fma(ps, u, -1.0 / 5040.0);           // 1/7!
  ps = fma(ps, u, 1.0 / 120.0);             // 1/5!
  ps = fma(ps, u, -1.0 / 6.0);              // 1/3!
  ps = fma(ps, u, 1.0);
  // cos r = sum_{n<=9} (-u)^n / (2n)!
  double pc = -1.0 / 6402373705728000.0;  // 1/18!
  pc = fma(pc, u, 1.0 / 20922789888000.0);  // 1/16!
  pc = fma(pc, u, -1.0 / 87178291200.0);    // 1/14!
  pc = fma(pc, u, 1.0 / 479001600.0);       // 1/12!
  pc = fma(pc, u, -1.0 / 3628800.0);        // 1/10!
  pc = fma(pc, u, 1.0 / 40320.0);           // 1/8!
  pc = fma(pc, u, -1.0 / 720.0);            // 1/6!
  pc = fma(pc, u, 1.0 / 24.0);              // 1/4!
  pc = fma(pc, u, -0.5);
  pc = fma(pc, u, 1.0);
  const double s0 = r * ps, c0 = pc;
  // x = k pi/2 + r: rotate (s0, c0) by the quadrant k mod 4
  const int q = (int)((long long)k & 3);
  const double a = (q & 1) ? c0 : s0;
  const double b = (q & 1) ? s0 : c0;
  *sn = (q & 2) ? -a : a;
  *cs = ((q + 1) & 2) ? -b : b;
}

// ----------------------------------------------------------------- potential
// w = U v for the complex-symmetric U given by its packed upper triangle
// (S(S+1)/2 entries, row-major); conj = 1 applies conj(U) = U(-tau).
template <typename T, int S>
__device__ __forceinline__ void apply_u(cx<T> (&w)[S], const cx<T> (&u)[S * (S + 1) / 2]) {
  cx<T> in[S];
#pragma unroll
  for (int s = 0; s < S; ++s) in[s] = w[s];
#pragma unroll
  for (int i = 0; i < S; ++i) {
    cx<T> acc = {(T)0, (T)0};
#pragma unroll
    for (int j = 0; j < S; ++j) {
      const int a = i < j ? i : j, b = i < j ? j : i;
      const int e = a * S - (a * (a - 1)) / 2 + (b - a);
      acc = cadd(acc, cmul(u[e], in[j]));
    }
    w[i] = acc;
  }
}

// w = U v for the complex-symmetric U given by its packed upper triangle
// (S(S+1)/2 entries, row-major) of factors read from a (split) table.  In
// FP32 the matvec runs in FP64 on U = rounded + residue (exact to about
// 1e-15) and each output is rounded to FP32 once.  An FP32 matvec would
// round its partial sums, and with a coupling the potential action is a
// near-identity unitary whose departure from the identity per step (the
// population moved between surfaces) is a few parts in 1e8: those roundings
// then lose norm at every action (measured on the two-surface model, 1000
// Strang steps: norm 1.9e-5 low; with one rounding per output the norm only
// wanders at the 1e-7 level).
template <typename T, int S>
__device__ __forceinline__ void apply_u_fac(cx<T> (&w)[S], const Fac<T> (&u)[S * (S + 1) / 2]) {
  if constexpr (!std::is_same<T, float>::value) {
    cx<T> uw[S * (S + 1) / 2];
#pragma unroll
    for (int e = 0; e < S * (S + 1) / 2; ++e) uw[e] = u[e].w;
    apply_u<T, S>(w, uw);
  } else {
    cx<double> ud[S * (S + 1) / 2];
#pragma unroll
    for (int e = 0; e < S * (S + 1) / 2; ++e)
      ud[e] = cx<double>{(double)u[e].w.re + (double)u[e].lo.re,
                         (double)u[e].w.im + (double)u[e].lo.im};
    cx<double> in[S];
#pragma unroll
    for (int s = 0; s < S; ++s) in[s] = cx<double>{(double)w[s].re, (double)w[s].im};
#pragma unroll
    for (int i = 0; i < S; ++i) {
      cx<double> acc = {0.0, 0.0};
#pragma unroll
      for (int j = 0; j < S; ++j) {
        const int a = i < j ? i : j, b = i < j ? j : i;
        acc = cadd(acc, cmul(ud[a * S - (a * (a - 1)) / 2 + (b - a)], in[j]));
      }
      w[i] = cx<float>{(float)acc.re, (float)acc.im};
    }
  }
}

}  // namespace sop
