// internal.hpp -- host-side interface between the planner / C ABI and the
// HIP kernel launchers.  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <map>
#include <string>
#include <vector>

#include "../../include/soprop.h"

namespace sop {

// Program of one time step: an alternating list of actions.  Entry =
// (op << 16) | table index, op 0 = potential, 1 = kinetic.
enum { OP_V = 0, OP_T = 1 };
inline int prog_entry(int op, int idx) { return (op << 16) | idx; }
inline int prog_op(int e) { return e >> 16; }
inline int prog_idx(int e) { return e & 0xffff; }

// Kernel kinds reported by the timing hook.
enum { KIND_ZPASS = 0, KIND_YPASS = 1, KIND_XPASS = 2, KIND_1D = 3, KIND_OTHER = 4, KIND_PLANE = 5,
       KIND_INTERP = 6, KIND_COUNT = 7 };

// Optional per-launch timing: HIP events recorded on the plan's stream
// between kernel launches, resolved after a synchronisation.  Consecutive
// timed launches share their boundary event (one event record per launch,
// not two), so the intervals of a run of launches tile its wall time; any
// untimed work on the stream must break the chain first.
struct Timer {
  struct Rec {
    int kind;
    hipEvent_t a, b;
    double bytes;
  };
  std::vector<Rec> recs;
  std::vector<hipEvent_t> pool;
  size_t used = 0;
  hipEvent_t last = nullptr;  // end event of the previous timed launch
  hipStream_t last_stream = nullptr;
  void break_chain() { last = nullptr; }
  hipEvent_t get() {
    if (used == pool.size()) {
      hipEvent_t e;
      if (hipEventCreate(&e) != hipSuccess) return nullptr;
      pool.push_back(e);
    }
    return pool[used++];
  }
  ~Timer() {
    for (hipEvent_t e : pool) (void)hipEventDestroy(e);
  }
};

// One pass of the 3D executor: Z = potential action(s), then (kz) the z
// factor of kinetic set tidx; Y, X = the y / x factor of set tidx; XY = both
// in one plane pass.
struct PassDesc {
  enum Kind { Z = 0, Y = 1, X = 2, XY = 3 };
  int kind = Z;
  bool kz = false;
  int nv = 0, iv0 = 0, iv1 = 0;  // z-pass potential actions
  int tidx = 0;                  // kinetic factor set
  bool operator==(const PassDesc& o) const {
    return kind == o.kind && kz == o.kz && nv == o.nv && iv0 == o.iv0 && iv1 == o.iv1 &&
           tidx == o.tidx;
  }
};

// Instantiated HIP graphs of step segments (first step, steady step, final
// flush), captured on a private stream and launched on the plan's stream.
struct GraphCache {
  struct Key {
    const void* psi;
    int conj, count, seg;
    bool operator<(const Key& o) const {
      if (psi != o.psi) return psi < o.psi;
      if (conj != o.conj) return conj < o.conj;
      if (count != o.count) return count < o.count;
      return seg < o.seg;
    }
  };
  hipStream_t capture = nullptr;
  std::map<Key, hipGraphExec_t> execs;
  void clear() {
    for (auto& kv : execs) (void)hipGraphExecDestroy(kv.second);
    execs.clear();
  }
  ~GraphCache() {
    clear();
    if (capture) (void)hipStreamDestroy(capture);
  }
};

// Device-side view of a plan that the launchers need.
struct DevView {
  int ndim = 1;
  int n[3] = {1, 1, 1};  // axis lengths, axis 0 slowest
  int S = 1;
  int64_t npts = 1;
  bool f64 = true;
  hipStream_t stream = nullptr;
  // [n_vtab][S(S+1)/2][npts] complex (FP32: (rounded, residue) pairs); when
  // `eig`, the one compact FP64 eigen-form table instead
  const void* vexp = nullptr;
  bool eig = false;
  const double* vtaus = nullptr;  // device c dt / hbar of each potential coefficient
  const void* kin = nullptr;   // 1D: [n_ttab][n0]; 3D: [n_ttab][3][kin_stride]
  int kin_stride = 0;          // complex entries per axis block (3D)
  const void* tw[3] = {nullptr, nullptr, nullptr};  // per-axis twiddles exp(-2 pi i k/n)
  const int* prog = nullptr;   // device copy of the step program
  int nact = 0;
  std::vector<int> hprog;      // host copy of the step program
  Timer* timer = nullptr;      // non-null while timing is enabled
  GraphCache* graphs = nullptr;  // non-null when 3D steps may be graph-captured
  int count = 1;               // states of a batch processed by each 3D launch
  bool plane = true;           // fused xy plane pass where the plane fits in LDS
};

// Brackets one launch with timing events when the plan's timer is on.
struct TimedLaunch {
  const DevView& d;
  Timer::Rec rec{};
  bool on;
  TimedLaunch(const DevView& dv, int kind, double bytes) : d(dv), on(dv.timer != nullptr) {
    if (on) {
      rec.kind = kind;
      rec.bytes = bytes;
      Timer& t = *d.timer;
      if (t.last && t.last_stream == d.stream) {
        rec.a = t.last;
      } else {
        rec.a = t.get();
        if (!rec.a || hipEventRecord(rec.a, d.stream) != hipSuccess) on = false;
      }
      rec.b = on ? t.get() : nullptr;
      if (!rec.b) on = false;
      if (!on) t.break_chain();
    }
  }
  ~TimedLaunch() {
    if (!on) return;
    if (hipEventRecord(rec.b, d.stream) == hipSuccess) {
      d.timer->recs.push_back(rec);
      d.timer->last = rec.b;
      d.timer->last_stream = d.stream;
    } else {
      d.timer->break_chain();
    }
  }
};

// kernels_1d.hip
bool k1d_supported(int n, int S);
// count states [count][S][N] of the same plan, one workgroup each
hipError_t k1d_propagate(const DevView& d, void* psi, int64_t nsteps, int conj, int count = 1);
hipError_t k1d_fft_forward(const DevView& d, void* psi);

// Device buffers of an adjoint sweep (FP64 only).
struct AdjointView {
  void* stacked = nullptr;      // [2S][npts] complex: psi then lambda
  const void* eig = nullptr;    // eigen form per point, z-pass tile layout: S >= 2 the
                                // compact form (eig_slots(S) slots), S = 1 the pair (1, V)
  double* qacc = nullptr;       // packed gradient accumulator, S(S+1)/2 doubles a point,
                                // [tile (y, x/C)][z][entry][x % C], C = k3d_adjoint_cols
  const double* taus = nullptr; // c dt / hbar of each potential table
  const void* checkpoints = nullptr;  // [ncp][S][npts] complex, psi at steps 0, K, 2K, ...
};

// kernels_3d.hip
bool k3d_supported(int n, int S);
bool k3d_adjoint_supported(int n, int S, bool f64);
// Columns per tile of the adjoint z-pass and of its gradient accumulator.
int k3d_adjoint_cols(int n);
hipError_t k3d_adjoint_backward(const DevView& d, const AdjointView& a, int64_t nsteps, int K);
// Columns per z-pass tile; 3D potential tables are stored tile-contiguous
// ([tile (y, x/C)][z][entry][x % C]) with this C.
int k3d_table_tile(int n, bool f64);
hipError_t k3d_propagate(const DevView& d, void* psi, int64_t nsteps, int conj);
bool k3d_plane(int n, bool f64);  // the xy plane of an n^3 grid fits in LDS
hipError_t k3d_fft_forward(const DevView& d, void* psi);

// Complex double slots per point of the compact eigen form (3D, S = 2, 3).
constexpr int eig_slots(int S) { return S == 3 ? 4 : 2; }
// Whether a plan of this kind can store the eigen form instead of
// per-coefficient tables (it does when every phase tau lam stays within
// kPhaseMax).  The form is FP64 in both precisions; FP32 plans apply it in
// FP64 and round the state once.
constexpr bool eig_form(int ndim, int S) { return ndim == 3 && S >= 2; }

// kernels_trap.hip: compositions of the trapezoidal rule on 1D FP64 plans,
// one workgroup per state (count states of S x N, consecutive).
struct TrapArgs {
  void* psi = nullptr;        // [count][S][N] complex, advanced in place
  void* rbuf = nullptr;       // [count][S][N] complex residual workspace
  const double* vraw = nullptr;  // [S(S+1)/2][N] V-table
  const double* taus = nullptr;  // [nst] g_j dt / (2 hbar)
  int nst = 0;
  int64_t nsteps = 0;
  double tk = 0;    // T(k) = tk * k^2 (k the signed frequency index)
  double tol2 = 0;  // squared relative residual at which a solve stops
  int maxit = 0;
  long long* stats = nullptr;  // [count][3]: iterations, failed stages, most iterations
  int count = 1;
};
bool k1d_trap_supported(int n, int S);
hipError_t k1d_trapezoid(const DevView& d, const TrapArgs& g);
// kernels_trap3d.hip: the trapezoidal rule on 3D FP64 plans (one state at a
// time).  x is the iterate (the state itself), r the residual, p the search
// direction, ap = A p; qz, qy, qx the three one-axis kinetic terms of H u
// (computed by the pass kernels, k3d_axis_kinetic, on copies of u);
// partials [kReduceBlocks][4] and sums [4] the reductions.
struct Trap3Bufs {
  void* x = nullptr;
  void* r = nullptr;
  void* p = nullptr;
  void* ap = nullptr;
  void* qz = nullptr;
  void* qy = nullptr;
  void* qx = nullptr;
  double* partials = nullptr;  // kT3Partials doubles
  double* sums = nullptr;      // the status block, kT3Status doubles (T3_*)
};
// Status block of the 3D trapezoidal iteration (doubles): |b|^2, rho =
// r^T r (re, im), mu = p^T A p (re, im), |r|^2, rho after the last update
// (re, im), the stop flag (converged, broken down or out of iterations),
// the iteration count, the breakdown flag, tol^2 and the iteration limit.
enum { T3_BB = 0, T3_RHO = 1, T3_MU = 3, T3_RR = 5, T3_RHO_NEW = 6, T3_STOP = 8, T3_ITER = 9,
       T3_FAIL = 10, T3_TOL2 = 11, T3_MAXIT = 12, kT3Status = 13 };
constexpr int kT3Partials = 9 * 1024;  // 9 x kReduceBlocks
// From x: r = p = -2 i tau H x; the status for a new stage.
hipError_t t3_init(const Trap3Bufs& b, int S, const double* vraw, int64_t npts, double tau,
                   double tol2, int max_iter, hipStream_t st);
// ap = p + i tau H p with its partial sums of p^T ap.
hipError_t t3_ap(const Trap3Bufs& b, int S, const double* vraw, int64_t npts, double tau,
                 hipStream_t st);
// x += alpha p, r -= alpha ap (alpha from the sums of t3_ap and of the last
// update); the iteration count.  parity: the iteration's index mod 2 (0 for
// the first iteration of a stage).
hipError_t t3_update(const Trap3Bufs& b, int S, int64_t npts, int parity, hipStream_t st);
// p = r + beta p; |r|^2 and the residual test, which freezes the status.
hipError_t t3_pupdate(const Trap3Bufs& b, int S, int64_t npts, int parity, hipStream_t st);
// One one-axis pass (axis 0 = slowest ("z"), 1, 2) of every surface:
// psi = F_a^-1 f_a F_a src (src NULL: psi itself) with the factor block of
// d.kin's set 0 for that axis (the propagator's pass kernels; no potential
// action).
hipError_t k3d_axis_kinetic(const DevView& d, void* psi, int axis, const void* src = nullptr);

// The allocation-free trapezoid call's static device scratch: its size, and
// its device address on the GPU of `stream` (NULL: the current device),
// looked up once per device and kept.
size_t trap_scratch_bytes();
hipError_t trap_scratch(hipStream_t stream, void** out);

// kernels_interp.hip: trigonometric interpolation between uniform grids.
// Complex FP64 product C[b] = A[b] B[b] (M x K by K x N) with element and
// batch strides; A needs sak = 1 or sai = 1, B sbj = 1 or sbk = 1.
struct CgemmArgs {
  const double2* A = nullptr;
  const double2* B = nullptr;
  double2* C = nullptr;
  int M = 0, N = 0, K = 0;
  long long sai = 0, sak = 0, sbk = 0, sbj = 0, sci = 0, scj = 0;
  long long bsa = 0, bsb = 0, bsc = 0;
};
// W [nd][n]: the interpolation matrix from the n-point grid on [lo, hi) to the
// nd-point grid on [lod, hid).
hipError_t interp_weights(hipStream_t s, double2* W, int n, double lo, double hi, int nd,
                          double lod, double hid);
hipError_t cgemm(hipStream_t s, const CgemmArgs& g, int batch);

// kernels_aux.hip
// tile = 0: [u][entry][point] (1D); tile = C: the z-pass tile layout (3D).
hipError_t form_vexp(const DevView& d, const double* vraw_dev, const double* taus, int ntau,
                     int tile, void* out,
                     const double* dtab = nullptr, const double* s_dev = nullptr);
hipError_t obs_reduce(const DevView& d, const void* psi, const void* psi_hat,
                      const double* vraw_dev, const double* inv_mass, const double* dx,
                      double hbar, double* partials_dev, double* out_dev);
hipError_t overlap_reduce(const DevView& d, const void* psi, const void* phi,
                          double* partials_dev, double* out_dev);
hipError_t distance_reduce(const DevView& d, const void* psi, const void* phi,
                          double* partials_dev, double* out_dev);
hipError_t form_eig(const DevView& d, const double* vraw_dev, int tile, void* out);
// compact eigen form, eig_slots(S) slots per point in the z-pass tile layout
hipError_t form_eigq(const DevView& d, const double* vraw_dev, int tile, void* out,
                     const double* dtab = nullptr, const double* s_dev = nullptr);
hipError_t set_vparams(const DevView& d, double* vraw, const double* vbase, const double* dv,
                       const double* delta_dev, int nparams);
hipError_t adjoint_seed(const DevView& d, void* lam, const void* psi, const double* w_dev,
                        double* qacc);
// qacc in the accumulator's tile layout with `cols` columns per tile
hipError_t grad_reduce(const DevView& d, const double* qacc, int cols, const double* dv,
                       int nparams, double* partials, double* out_dev);
// out_dev[0..S) = sum |psi_s|^2, out_dev[S] = sum psi^dag V psi (raw sums)
hipError_t pops_reduce(const DevView& d, const void* psi, const double* vraw_dev,
                       double* partials, double* out_dev);
// ------------------------------------------------------------------ batches
// Device descriptor of one 1D member of a batch (kernels_batch1d.hip).
struct BMember1 {
  void* psi;          // [S][N]
  const void* vexp;   // [n_vtab][S(S+1)/2][N]
  const void* kin;    // [n_ttab][N]
  const void* tw;     // [N] twiddles
  const int* prog;    // step program
  int64_t nsteps;
  int nact;
  int conj;
};
// Device descriptor of one 3D member of a lockstep group
// (kernels_batch3d.hip).  The member's program is the pruned VTV sequence
// V T V ... T V (nact = 2M + 1); cycle c < cycles = M * nsteps is its
// kinetic action number c with the potential action(s) before it, cycle
// c = cycles its closing potential action.
struct BMember3 {
  void* psi;          // [S][n^3]
  const void* vexp;   // tile-layout potential tables (or the FP64 eigen form, S >= 2)
  const double* vtaus;  // c dt / hbar of each potential coefficient (eigen form)
  const void* kin;    // [n_ttab][3][kin_stride]
  const void* tw;     // [3][n] twiddles (z, y, x blocks)
  const int* prog;
  int64_t cycles;
  int M;
  int conj;
  int kin_stride;
  int pad;
};

// plan.cpp: the device view of a plan, and the thread-local error text that
// sop_last_error returns.
const DevView* plan_view(const sop_plan* p);
void set_last_error(const std::string& msg);

// 1D families: candidate schedules ("variants") of each length; variant 0 is
// the schedule of the single-plan kernel.
int k1b_variants(int n, int S);
const char* k1b_variant_name(int n, int S, int variant, bool f64);
// Runs members mem[0..count) (one workgroup each, in order) with the variant.
hipError_t k1b_launch(int n, int S, bool f64, int variant, const BMember1* mem, int count,
                      hipStream_t stream);

// 3D lockstep groups.  kind: 0 z-pass (potential, z factor), 1 y factor,
// 2 x factor, 3 fused xy plane (kinds 1 and 2 in one pass, where the plane
// fits in LDS).
enum { B3_Z = 0, B3_Y = 1, B3_X = 2, B3_XY = 3 };
bool k3b_supported(int n, int S);
bool k3b_plane(int n, bool f64);
int k3b_variants(int kind, int n, bool f64);
int k3b_variant_width(int kind, int n, bool f64, int variant);  // columns or rows per tile
hipError_t k3b_launch(int kind, int n, int S, bool f64, int variant, const BMember3* mem,
                      int count, int64_t cycle, hipStream_t stream);

// 3D groups as one work-queue launch (kernels_batch3d.hip).  Round p of a
// group is pass number p of every member still running then: p = 3c the
// z-pass of cycle c (the closing one where c = cycles), 3c + 1 and 3c + 2
// its y- and x-passes.  Every member's work items are numbered by its own
// ticket counter, round after round: round p's items are tickets
// [need, next round's need), and an item of round p may start once its
// member has finished `need` items (all of rounds 0..p-1); a member with c
// cycles runs rounds 0..3c.  The members, in decreasing order of cycles,
// run in round p while their index is below `members`, and start counts
// the group's items before round p (both for the description only).
// rounds[nrounds] is a sentinel round.
struct QRound {
  int64_t start;
  int64_t need;
  int64_t cycle;
  int kind;     // B3_Z, B3_Y or B3_X
  int members;
};
// Control block of a queue launch, one 64-bit word per 256-byte slot (the
// counters that many waves poll or add to do not share a cache line):
// slot 1 the abort flag (a wait ran out of polls; every wave leaves), slot 2
// a sticky copy of it (cleared only by the host), slot 3 + m the items
// member m has finished, slot 3 + members + m its next ticket.
constexpr int kQCtrlHead = 3;
constexpr int kQSlot = 32;  // words per slot
constexpr size_t q_ctrl_words(int members) {
  return (size_t)(kQCtrlHead + 2 * members) * kQSlot;
}
bool k3q_supported(int n, int S);
int k3q_tiles(int kind, int n, int S, bool f64);  // work items of one member in a round
// Persistent workgroups a queue launch uses (occupancy x compute units).
int k3q_grid(int n, int S, bool f64);
// Clears the control block (all but the sticky flag), then runs the queue.
// The control block must hold q_ctrl_words(count) words.
hipError_t k3q_launch(int n, int S, bool f64, const BMember3* mem, int count,
                      const QRound* rounds, int nrounds, int64_t tickets,
                      unsigned long long* ctrl, long long spin_limit, hipStream_t stream);

constexpr int kMaxParams = 8;
constexpr int kReduceBlocks = 1024;
static_assert(kT3Partials == 9 * kReduceBlocks, "trapezoid partial buffers");
constexpr int kReduceThreads = 256;

}  // namespace sop
