// kernels_batch3d.hip -- three-dimensional members of a batch: lockstep
// passes over every member of one (n, surfaces, precision) group.
//
// Each member runs the pruned VTV step program V(a_1) T(b_1) ... T(b_M)
// V(a_{M+1}) of its own plan (own order, dt, tables and step count).  Its
// pass sequence is periodic: cycle c (c < cycles = M nsteps) is the z-pass
// that applies the potential action(s) before kinetic action number c and
// that action's z factor, then the y- and x-passes (or the plane pass) of
// that kinetic action; the z-pass of cycle c = cycles applies the closing
// V(a_{M+1}).  At a step boundary the z-pass applies V(a_{M+1}) of the
// finished step and V(a_1) of the next one (the same actions the
// single-plan executor launches).  Launch c of a kind covers every member; a
// member derives its own pass parameters from c and its program on the
// device, and members whose run is shorter than c leave at once.  The pass
// bodies are those of the single-plan kernels, so a member's result equals
// its single-plan run.
#include <algorithm>

#include "passes_3d.hpp"

namespace sop {
namespace {

using namespace s3d;

constexpr int prog_index(int code) { return code & 0xffff; }

// kinetic factor set of cycle c (c < cycles), axis a (0 z, 1 y, 2 x)
template <typename T>
__device__ __forceinline__ const cx<T>* cycle_kin(const BMember3& m, int64_t c, int a) {
  const int tidx = prog_index(m.prog[2 * (int)(c % m.M) + 1]);
  return (const cx<T>*)m.kin + ((size_t)tidx * 3 + a) * m.kin_stride;
}

// z-pass of cycle c: grid (N / C, N, members)
template <typename T, class SC, int S, int C>
__global__ void __launch_bounds__(C * SC::TPC)
    k3b_zpass(const BMember3* __restrict__ mem, int64_t c) {
  extern __shared__ char smem_raw[];
  cx<T>* lds = reinterpret_cast<cx<T>*>(smem_raw);
  const BMember3 m = mem[blockIdx.z];
  if (m.cycles <= 0 || c > m.cycles) return;
  const int M = m.M;
  cx<T>* psi = (cx<T>*)m.psi;
  const void* vexp = m.vexp;
  const cx<T>* tw = (const cx<T>*)m.tw;
  constexpr bool EQ = eig_form(3, S);
  if (c == m.cycles) {  // closing potential action
    zpass_body<T, SC, S, C, kTableCols, AX_NONE, EQ>(psi, vexp, 1, prog_index(m.prog[2 * M]),
                                                     0, m.conj, tw, nullptr, lds, blockIdx.x,
                                                     blockIdx.y, m.vtaus);
    return;
  }
  const int i = (int)(c % M);
  int nv = 1, iv0 = prog_index(m.prog[2 * i]), iv1 = 0;
  if (c > 0 && i == 0) {  // step boundary: V(a_{M+1}) then V(a_1)
    nv = 2;
    iv0 = prog_index(m.prog[2 * M]);
    iv1 = prog_index(m.prog[0]);
  }
  zpass_body<T, SC, S, C, kTableCols, AX_KIN, EQ>(psi, vexp, nv, iv0, iv1, m.conj, tw,
                                                  cycle_kin<T>(m, c, 0), lds, blockIdx.x,
                                                  blockIdx.y, m.vtaus);
}

// y-pass of cycle c: grid (N / C, N, S x members).
template <typename T, class SC, int C>
__global__ void __launch_bounds__(C * SC::TPC)
    k3b_ypass(const BMember3* __restrict__ mem, int S, int64_t c) {
  extern __shared__ char smem_raw[];
  cx<T>* lds = reinterpret_cast<cx<T>*>(smem_raw);
  const int mi = blockIdx.z / S, s = blockIdx.z % S;
  const BMember3 m = mem[mi];
  if (c >= m.cycles) return;
  constexpr int64_t npts = (int64_t)SC::N * SC::N * SC::N;
  const cx<T>* tw = (const cx<T>*)m.tw + SC::N * Split<T>::rep;  // the y block
  ypass_body<T, SC, C, AX_KIN>((cx<T>*)m.psi + s * npts, tw, cycle_kin<T>(m, c, 1), m.conj, lds,
                               blockIdx.x, blockIdx.y);
}

// x-pass of cycle c: grid (N / ROWS, N, S x members).
template <typename T, class SC, int ROWS>
__global__ void __launch_bounds__(ROWS * SC::TPC)
    k3b_xpass(const BMember3* __restrict__ mem, int S, int64_t c) {
  extern __shared__ char smem_raw[];
  cx<T>* lds = reinterpret_cast<cx<T>*>(smem_raw);
  const int mi = blockIdx.z / S, s = blockIdx.z % S;
  const BMember3 m = mem[mi];
  if (c >= m.cycles) return;
  constexpr int64_t npts = (int64_t)SC::N * SC::N * SC::N;
  const cx<T>* tw = (const cx<T>*)m.tw + 2 * SC::N * Split<T>::rep;  // the x block
  xpass_body<T, SC, ROWS, AX_KIN>((cx<T>*)m.psi + s * npts, tw, cycle_kin<T>(m, c, 2), m.conj,
                                  lds, blockIdx.x, blockIdx.y);
}

// fused xy plane pass of cycle c: grid (N planes, S x members).
template <typename T, class SC>
__global__ void __launch_bounds__(SC::N * SC::TPC)
    k3b_plane(const BMember3* __restrict__ mem, int S, int64_t c) {
  extern __shared__ char smem_raw[];
  cx<T>* lds = reinterpret_cast<cx<T>*>(smem_raw);
  const int mi = blockIdx.y / S, s = blockIdx.y % S;
  const BMember3 m = mem[mi];
  if (c >= m.cycles) return;
  constexpr int64_t npts = (int64_t)SC::N * SC::N * SC::N;
  plane_body<T, SC>((cx<T>*)m.psi + s * npts, (const cx<T>*)m.tw, cycle_kin<T>(m, c, 0),
                    m.conj, lds, blockIdx.x);
}

// ---------------------------------------------------------------- work queue
// One persistent launch runs every pass of every member of a group.  The
// pass tiles are one wave each: a z-pass tile of W columns, a y-pass tile
// of W columns or an x-pass tile of W rows of one surface plane,
// W = 64 / (threads per pencil).  A work item is kQWaves consecutive tiles
// of one member's pass, run side by side by the waves of one workgroup.
// Every member numbers its items with its own ticket counter, round after
// round (QRound).  A workgroup serves one member at a time, starting with
// member blockIdx.x mod count: it takes the member's next ticket, waits
// until the member has finished every item of the earlier rounds (the
// member's completion counter reaches the round's `need`), runs its tiles
// with the same pass bodies as the lockstep kernels, and adds one to the
// completion counter after its stores.  It takes the member's next ticket
// before working on the current one, so the counter's latency hides behind
// the item; once the member's tickets run out it finishes the item, then
// moves on to the next member with tickets left, and leaves when none has
// any.  Items of several tiles and one counter pair per member keep the
// counter traffic down: same-address atomics are served one at a time.
//
// Progress: a workgroup holds tickets only while it runs, all of one member,
// works on them in increasing order, and waits only for smaller tickets of
// that member, so the holder of a member's smallest unfinished ticket never
// waits; nothing assumes that the grid is resident at once.
// Waits are bounded by spin_limit polls: a wait that runs out raises the
// abort flag, and every wave that sees it leaves (the host reports it).
constexpr int kQWaves = 4;
constexpr int kQThreads = 64 * kQWaves;

template <class SC>
constexpr int qwidth() {
  return 64 / SC::TPC;
}
// LDS elements of one tile (the largest pass kind)
template <typename T, class SC>
constexpr size_t q_tile_elems() {
  constexpr int W = qwidth<SC>(), N = SC::N;
  constexpr size_t z = (size_t)W * N, y = y_lds_elems<T, N>(W), x = x_lds_elems<T, N>(W);
  return z > y ? (z > x ? z : x) : (y > x ? y : x);
}
template <typename T, class SC>
constexpr size_t q_lds_bytes() {
  return kQWaves * q_tile_elems<T, SC>() * sizeof(cx<T>);
}

template <typename T, class SC, int S>
__global__ void __launch_bounds__(kQThreads)
    k3q_run(const BMember3* __restrict__ mem, int count, const QRound* __restrict__ rounds,
            int nrounds, unsigned long long* __restrict__ ctrl, long long spin_limit) {
  static_assert(64 % SC::TPC == 0 && SC::N % qwidth<SC>() == 0, "tile shape");
  extern __shared__ char smem_raw[];
  constexpr int N = SC::N, W = qwidth<SC>(), NB = N / W;
  constexpr int TZ = NB * N, TYX = NB * N * S;  // tiles of one member in a round
  static_assert(TZ % kQWaves == 0, "items of whole tiles");
  const int wave = (int)threadIdx.x / 64;
  cx<T>* lds = reinterpret_cast<cx<T>*>(smem_raw) + (size_t)wave * q_tile_elems<T, SC>();
  constexpr int64_t npts = (int64_t)N * N * N;
  constexpr int A = axis_block<T, N>();
  constexpr bool EQ = eig_form(3, S);
  const int lane = (int)threadIdx.x % 64;
  const bool lead = threadIdx.x == 0;
  __shared__ long long bcast[2];
  unsigned long long* const abort_flag = ctrl + kQSlot;
  unsigned long long* const done = ctrl + kQCtrlHead * kQSlot;            // member m at m * kQSlot
  unsigned long long* const next = ctrl + (kQCtrlHead + count) * kQSlot;  // likewise
  // the leader takes member mi's next ticket (tickets past the member's
  // last item mean none)
  auto claim = [&](int mi) -> long long {
    return (long long)__hip_atomic_fetch_add(next + (size_t)mi * kQSlot, 1ull, __ATOMIC_RELAXED,
                                             __HIP_MEMORY_SCOPE_AGENT);
  };
  auto last = [&](int mi) -> long long {  // the member's ticket count
    const int64_t cy = mem[mi].cycles;
    return cy > 0 ? rounds[3 * cy + 1].need : 0;
  };
  // find a member with tickets left, starting at mi; -1: none left
  auto find = [&](int mi, long long* tk) -> int {
    for (int k = 0; k < count; ++k, mi = (mi + 1) % count) {
      const long long v = claim(mi);
      if (v < last(mi)) {
        *tk = v;
        return mi;
      }
    }
    return -1;
  };
  if (lead) {
    long long t0 = 0;
    const int m0 = find((int)(blockIdx.x % (unsigned)count), &t0);
    bcast[0] = m0;
    bcast[1] = t0;
  }
  __syncthreads();
  int mi = (int)bcast[0];
  long long t = bcast[1];
  __syncthreads();  // every wave has read them before the leader writes again
  int p = 0;
  while (mi >= 0) {
    while (t >= rounds[p + 1].need) ++p;
    const QRound r = rounds[p];
    const int tile = (int)(t - r.need) * kQWaves + wave;
    // the leader's next ticket of this member (-1: none left; another
    // member's ticket is taken only once this item is done, so a workgroup
    // never holds tickets of two members)
    long long tn = 0;
    if (lead) {
      tn = claim(mi);
      if (tn >= last(mi)) tn = -1;
    }
    // wait until the member has finished the earlier rounds
    unsigned ok = 1;
    unsigned long long* const cnt = done + (size_t)mi * kQSlot;
    if (lead) {
      long long polls = 0;
      int backoff = 1;  // s_sleep(1) units between polls, doubling to 32 (about 1 us)
      while ((long long)__hip_atomic_load(cnt, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) <
             r.need) {
        if (__hip_atomic_load(abort_flag, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0 ||
            ++polls > spin_limit) {
          ok = 0;
          break;
        }
        for (int k = 0; k < backoff; ++k) __builtin_amdgcn_s_sleep(1);
        backoff = backoff < 32 ? 2 * backoff : 32;
      }
      if (!ok) {
        __hip_atomic_store(abort_flag, 1ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __hip_atomic_store(ctrl + 2 * kQSlot, 1ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      }
      // the member's earlier stores are visible to this workgroup's loads
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
      bcast[0] = ok;
      bcast[1] = tn;
    }
    __syncthreads();
    const bool go = bcast[0] != 0;
    long long tn_all = bcast[1];
    if (!go) break;
    const BMember3 m = mem[mi];
    const int64_t c = r.cycle;
    const int ln = opaque(lane);  // recomputed each item: see zpass_body
    cx<T>* psi = (cx<T>*)m.psi;
    const cx<T>* tw = (const cx<T>*)m.tw;
    if (r.kind == B3_Z) {
      const int bx = tile % NB, by = tile / NB;
      const int M = m.M;
      if (c == m.cycles) {  // closing potential action
        zpass_body<T, SC, S, W, kTableCols, AX_NONE, EQ>(psi, m.vexp, 1,
                                                         prog_index(m.prog[2 * M]), 0, m.conj,
                                                         tw, nullptr, lds, bx, by, m.vtaus, ln);
      } else {
        const int i = (int)(c % M);
        int nv = 1, iv0 = prog_index(m.prog[2 * i]), iv1 = 0;
        if (c > 0 && i == 0) {  // step boundary: V(a_{M+1}) then V(a_1)
          nv = 2;
          iv0 = prog_index(m.prog[2 * M]);
          iv1 = prog_index(m.prog[0]);
        }
        zpass_body<T, SC, S, W, kTableCols, AX_KIN, EQ>(psi, m.vexp, nv, iv0, iv1, m.conj, tw,
                                                        cycle_kin<T>(m, c, 0), lds, bx, by,
                                                        m.vtaus, ln);
      }
    } else {
      const int s = tile / TZ, rem = tile % TZ;
      const int bx = rem % NB, z = rem / NB;
      if (r.kind == B3_Y)
        ypass_body<T, SC, W, AX_KIN>(psi + s * npts, tw + A, cycle_kin<T>(m, c, 1), m.conj, lds,
                                     bx, z, ln);
      else
        xpass_body<T, SC, W, AX_KIN>(psi + s * npts, tw + 2 * A, cycle_kin<T>(m, c, 2), m.conj,
                                     lds, bx, z, ln);
    }
    // every wave's stores are visible device-wide before the counter moves
    // (workgroup-scope release at the barrier, then the leader's release at
    // agent scope; the broadcast was read before this barrier, so the
    // leader may write it again afterwards)
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
    __syncthreads();
    if (lead) {
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
      __hip_atomic_fetch_add(cnt, 1ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    if (tn_all >= 0) {
      t = tn_all;
      continue;
    }
    // this member has no tickets left: the next member that has
    if (lead) {
      long long t1 = 0;
      bcast[0] = find((mi + 1) % count, &t1);
      bcast[1] = t1;
    }
    __syncthreads();
    const int mn = (int)bcast[0];
    tn_all = bcast[1];
    __syncthreads();  // read before the leader writes again
    if (mn < 0) break;
    int lo = 0, hi = nrounds;  // the ticket's round: rounds[lo].need <= t < rounds[hi].need
    while (hi - lo > 1) {
      const int mid = (lo + hi) / 2;
      if (rounds[mid].need <= tn_all)
        lo = mid;
      else
        hi = mid;
    }
    p = lo;
    mi = mn;
    t = tn_all;
  }
}

__global__ void k3q_clear(unsigned long long* __restrict__ ctrl, int count) {
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < kQCtrlHead + 2 * count;
       i += gridDim.x * blockDim.x)
    if (i != 2) ctrl[(size_t)i * kQSlot] = 0;  // the sticky flag stays
}

template <typename T, class SC, int S>
int q_grid() {
  static int cached = 0;
  if (cached > 0) return cached;
  int dev = 0, cus = 0, per = 0;
  if (hipGetDevice(&dev) != hipSuccess ||
      hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
      hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, k3q_run<T, SC, S>, kQThreads,
                                                   q_lds_bytes<T, SC>()) != hipSuccess) {
    (void)hipGetLastError();
    return 256;
  }
  cached = std::max(1, per) * std::max(1, cus);
  return cached;
}

template <typename T, class SC, int S>
hipError_t q_launch(const BMember3* mem, int count, const QRound* rounds, int nrounds,
                    int64_t tickets, unsigned long long* ctrl, long long spin_limit,
                    hipStream_t st) {
  hipLaunchKernelGGL(k3q_clear, dim3(1), dim3(256), 0, st, ctrl, count);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess || tickets <= 0) return e;
  auto k = k3q_run<T, SC, S>;
  const int grid = q_grid<T, SC, S>();
  const size_t lds = q_lds_bytes<T, SC>();
  hipLaunchKernelGGL(k, dim3(grid), dim3(kQThreads), lds, st, mem, count, rounds, nrounds, ctrl,
                     spin_limit);
  return hipGetLastError();
}

template <typename T, class SC, class F>
hipError_t by_surfaces(int S, F&& f) {
  switch (S) {
    case 1: return f.template operator()<T, SC, 1>();
    case 2: return f.template operator()<T, SC, 2>();
    case 3: return f.template operator()<T, SC, 3>();
    default: return hipErrorInvalidValue;
  }
}

// ---------------------------------------------------------------- variants
// z: pass tile of 16 or 8 columns (the table tile is 16 wide).
constexpr int zwidth(int v) { return v == 0 ? kTableCols : kTableCols / 2; }
// y: default columns, twice, half; x: default rows, twice, half.
constexpr int scaled(int base, int v) { return v == 0 ? base : (v == 1 ? 2 * base : base / 2); }

template <class SC, typename T>
constexpr int ywidth(int v) {
  return scaled(cols<SC, T>(), v);
}
template <class SC>
constexpr int xwidth(int v) {
  return scaled(xrows<SC>(), v);
}
template <class SC>
constexpr bool valid_width(int w) {
  return w >= 1 && SC::N % w == 0 && w * SC::TPC <= 1024 && w * SC::TPC >= 32;
}

template <typename K>
hipError_t set_lds(K k, size_t bytes) {
  if (bytes <= 64 * 1024) return hipSuccess;
  return hipFuncSetAttribute((const void*)k, hipFuncAttributeMaxDynamicSharedMemorySize,
                             (int)bytes);
}

template <typename T, class SC, int S, int V>
hipError_t launch_z(const BMember3* mem, int count, int64_t c, hipStream_t st) {
  constexpr int C = zwidth(V);
  const size_t lds = (size_t)C * SC::N * sizeof(cx<T>);
  auto k = k3b_zpass<T, SC, S, C>;
  hipError_t e = set_lds(k, lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k, dim3(SC::N / C, SC::N, count), dim3(C * SC::TPC), lds, st, mem, c);
  return hipGetLastError();
}

template <typename T, class SC, int V>
hipError_t launch_y(int S, const BMember3* mem, int count, int64_t c, hipStream_t st) {
  constexpr int C = ywidth<SC, T>(V);
  if constexpr (!valid_width<SC>(C)) {
    return hipErrorInvalidValue;
  } else {
    const size_t lds = y_lds_elems<T, SC::N>(C) * sizeof(cx<T>);
    auto k = k3b_ypass<T, SC, C>;
    hipError_t e = set_lds(k, lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k, dim3(SC::N / C, SC::N, S * count), dim3(C * SC::TPC), lds, st, mem, S,
                       c);
    return hipGetLastError();
  }
}

template <typename T, class SC, int V>
hipError_t launch_x(int S, const BMember3* mem, int count, int64_t c, hipStream_t st) {
  constexpr int R = xwidth<SC>(V);
  if constexpr (!valid_width<SC>(R)) {
    return hipErrorInvalidValue;
  } else {
    auto k = k3b_xpass<T, SC, R>;
    const size_t lds = x_lds_elems<T, SC::N>(R) * sizeof(cx<T>);
    hipError_t e = set_lds(k, lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k, dim3(SC::N / R, SC::N, S * count), dim3(R * SC::TPC), lds, st, mem, S,
                       c);
    return hipGetLastError();
  }
}

template <typename T, class SC>
hipError_t launch_plane(int S, const BMember3* mem, int count, int64_t c, hipStream_t st) {
  if constexpr (!plane_fits<T, SC>()) {
    return hipErrorInvalidValue;
  } else {
    auto k = k3b_plane<T, SC>;
    const size_t lds = plane_lds_elems<T, SC>() * sizeof(cx<T>);
    hipError_t e = set_lds(k, lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k, dim3(SC::N, S * count), dim3(SC::N * SC::TPC), lds, st, mem, S, c);
    return hipGetLastError();
  }
}

template <typename T, class SC>
hipError_t launch_kind(int kind, int S, int v, const BMember3* mem, int count, int64_t c,
                       hipStream_t st) {
  switch (kind) {
    case B3_XY:
      return v == 0 ? launch_plane<T, SC>(S, mem, count, c, st) : hipErrorInvalidValue;
    case B3_Z: {
      auto z = [&]<int V>() -> hipError_t {
        if (S == 1) return launch_z<T, SC, 1, V>(mem, count, c, st);
        if (S == 2) return launch_z<T, SC, 2, V>(mem, count, c, st);
        if (S == 3) return launch_z<T, SC, 3, V>(mem, count, c, st);
        return hipErrorInvalidValue;
      };
      if (v == 0) return z.template operator()<0>();
      if (v == 1) return z.template operator()<1>();
      return hipErrorInvalidValue;
    }
    case B3_Y:
      if (v == 0) return launch_y<T, SC, 0>(S, mem, count, c, st);
      if (v == 1) return launch_y<T, SC, 1>(S, mem, count, c, st);
      if (v == 2) return launch_y<T, SC, 2>(S, mem, count, c, st);
      return hipErrorInvalidValue;
    case B3_X:
      if (v == 0) return launch_x<T, SC, 0>(S, mem, count, c, st);
      if (v == 1) return launch_x<T, SC, 1>(S, mem, count, c, st);
      if (v == 2) return launch_x<T, SC, 2>(S, mem, count, c, st);
      return hipErrorInvalidValue;
    default:
      return hipErrorInvalidValue;
  }
}

template <class F>
hipError_t by_grid(int n, bool f64, F&& f) {
  switch (n) {
    case 32: return f64 ? f.template operator()<double, Z32>() : f.template operator()<float, Z32>();
    case 48: return f64 ? f.template operator()<double, Z48>() : f.template operator()<float, Z48>();
    case 64: return f64 ? f.template operator()<double, Z64>() : f.template operator()<float, Z64>();
    default: return hipErrorInvalidValue;
  }
}

// widths of the variants (0 if the variant does not exist)
template <typename T, class SC>
int width_of(int kind, int v) {
  if (kind == B3_XY) return (v == 0 && plane_fits<T, SC>()) ? SC::N : 0;
  if (kind == B3_Z) return (v == 0 || v == 1) ? zwidth(v) : 0;
  if (v < 0 || v > 2) return 0;
  const int w = (kind == B3_X) ? scaled(xrows<SC>(), v) : scaled(cols<SC, T>(), v);
  const bool ok = w >= 1 && SC::N % w == 0 && w * SC::TPC <= 1024 && w * SC::TPC >= 32;
  return ok ? w : 0;
}

}  // namespace

bool k3q_supported(int n, int S) { return (n == 32 || n == 48 || n == 64) && S >= 1 && S <= 3; }

int k3q_tiles(int kind, int n, int S, bool f64) {
  int r = 0;
  (void)by_grid(n, f64, [&]<typename T, class SC>() -> hipError_t {
    constexpr int NB = SC::N / qwidth<SC>();
    r = (kind == B3_Z ? NB * SC::N : NB * SC::N * S) / kQWaves;
    return hipSuccess;
  });
  return r;
}

int k3q_grid(int n, int S, bool f64) {
  int r = 0;
  (void)by_grid(n, f64, [&]<typename T, class SC>() -> hipError_t {
    return by_surfaces<T, SC>(S, [&]<typename T2, class SC2, int S2>() -> hipError_t {
      r = q_grid<T2, SC2, S2>();
      return hipSuccess;
    });
  });
  return r;
}

hipError_t k3q_launch(int n, int S, bool f64, const BMember3* mem, int count,
                      const QRound* rounds, int nrounds, int64_t tickets,
                      unsigned long long* ctrl, long long spin_limit, hipStream_t stream) {
  if (!k3q_supported(n, S) || count < 1 || spin_limit < 1) return hipErrorInvalidValue;
  return by_grid(n, f64, [&]<typename T, class SC>() -> hipError_t {
    return by_surfaces<T, SC>(S, [&]<typename T2, class SC2, int S2>() -> hipError_t {
      return q_launch<T2, SC2, S2>(mem, count, rounds, nrounds, tickets, ctrl, spin_limit,
                                   stream);
    });
  });
}

bool k3b_supported(int n, int S) { return (n == 32 || n == 48 || n == 64) && S >= 1 && S <= 3; }

int k3b_variant_width(int kind, int n, bool f64, int variant) {
  int w = 0;
  (void)by_grid(n, f64, [&]<typename T, class SC>() -> hipError_t {
    w = width_of<T, SC>(kind, variant);
    return hipSuccess;
  });
  return w;
}

int k3b_variants(int kind, int n, bool f64) {
  (void)n;
  (void)f64;
  return kind == B3_XY ? 1 : (kind == B3_Z ? 2 : 3);
}

bool k3b_plane(int n, bool f64) { return k3b_variant_width(B3_XY, n, f64, 0) > 0; }

hipError_t k3b_launch(int kind, int n, int S, bool f64, int variant, const BMember3* mem,
                      int count, int64_t cycle, hipStream_t stream) {
  if (count <= 0) return hipSuccess;
  if (k3b_variant_width(kind, n, f64, variant) == 0) return hipErrorInvalidValue;
  return by_grid(n, f64, [&]<typename T, class SC>() -> hipError_t {
    return launch_kind<T, SC>(kind, S, variant, mem, count, cycle, stream);
  });
}

}  // namespace sop
