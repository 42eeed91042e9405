// batch.cpp -- sop_batch: many independent plans propagated by one HIP graph.
//
// Members are grouped by the kernel that can run them together:
//   * 1D families (grid length, surfaces, precision): one persistent launch,
//     one workgroup per member for its whole run, members in decreasing
//     order of work;
//   * 3D lockstep groups (n in {32, 48, 64}, surfaces, precision, VTV
//     program): three pass launches per cycle, two with the plane pass
//     (kernels_batch3d.hip).  The members are sorted by decreasing cycle
//     count and cut into chains whose counts lie within a factor of 4 of
//     the chain's longest; each chain is its own branch, so a few long runs
//     proceed beside the bulk instead of after it, and launch c of a chain
//     covers only the members still running at cycle c;
//   * any other member runs its own plan's executor.
// Every family, group and single member is one branch of a fork/join HIP
// graph (branches on separate capture streams), so one propagate call is
// one graph launch; the graph is kept while the state pointers, step counts
// and direction stay the same.
//
// Tuning: at creation every family with several schedule variants and every
// lockstep group times its variants on scratch states with the members' own
// tables and keeps the fastest (z, y, x tiles of 3D groups chosen pass by
// pass).  SOPROP_TUNE=0 keeps the default variants; SOPROP_TUNE_CACHE=<path>
// reads choices from and adds new ones to a JSON file of "key": "variant"
// pairs.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <fstream>
#include <map>
#include <new>
#include <sstream>
#include <string>
#include <vector>

#include "../../include/soprop.h"
#include "internal.hpp"

using sop::BMember1;
using sop::BMember3;
using sop::DevView;

namespace {

// Largest graph (kernel nodes) a propagate call captures; longer runs are
// launched eagerly on the same branch streams.
constexpr int64_t kGraphNodeCap = 200000;
constexpr int kMaxBranches = 12;

sop_status fail(sop_status s, const std::string& msg) {
  sop::set_last_error(msg);
  return s;
}

#define HIPTRY(expr)                                                                 \
  do {                                                                               \
    hipError_t _e = (expr);                                                          \
    if (_e != hipSuccess) {                                                          \
      return fail(SOP_ERR_HIP, std::string(#expr) + ": " + hipGetErrorString(_e));   \
    }                                                                                \
  } while (0)

struct Family1 {
  int n = 0, S = 0;
  bool f64 = true;
  std::vector<int> members;
  int variant = 0;
  std::vector<double> tuned_ms;  // per variant (empty when not timed)
  bool from_cache = false;
  BMember1* d_mem = nullptr;
};

struct Group3 {
  int n = 0, S = 0;
  bool f64 = true;
  std::vector<int> members;
  int vz = 0, vy = 0, vx = 0;
  std::vector<double> ms_z, ms_y, ms_x;
  bool from_cache = false;
  BMember3* d_mem = nullptr;
  int64_t max_cycles = 0;
  // members sorted by decreasing cycle count; chains = contiguous ranges of
  // similar counts, each launched on its own branch
  std::vector<int64_t> cycles;
  std::vector<std::pair<int, int>> chains;
  // work-queue launch: round table (device copy and capacity in rounds),
  // ticket count, control block
  sop::QRound* d_rounds = nullptr;
  size_t rounds_cap = 0;
  int64_t nrounds = 0, tickets = 0;
  unsigned long long* d_ctrl = nullptr;
};

// Round table of a work-queue launch (sop::QRound) over the members of a
// group with cycle counts cyc[] in decreasing order (0: not running): z
// rounds hold the members with c <= cycles, y and x rounds those with
// c < cycles; tz and tyx are one member's tiles in a z and in a y or x
// round.  Appends the sentinel round and returns the ticket count.
int64_t build_rounds(const std::vector<int64_t>& cyc, int tz, int tyx,
                     std::vector<sop::QRound>& out) {
  out.clear();
  int nz = 0;
  while (nz < (int)cyc.size() && cyc[nz] > 0) ++nz;
  int nyx = nz;
  const int64_t cmax = nz > 0 ? cyc[0] : 0;
  int64_t start = 0, need = 0;
  auto push = [&](int64_t c, int kind, int k, int tiles) {
    out.push_back(sop::QRound{start, need, c, kind, k});
    start += (int64_t)k * tiles;
    need += tiles;
  };
  for (int64_t c = 0; nz > 0 && c <= cmax; ++c) {
    while (nz > 0 && cyc[nz - 1] < c) --nz;
    push(c, sop::B3_Z, nz, tz);
    if (c == cmax) break;
    while (nyx > 0 && cyc[nyx - 1] <= c) --nyx;
    push(c, sop::B3_Y, nyx, tyx);
    push(c, sop::B3_X, nyx, tyx);
  }
  out.push_back(sop::QRound{start, need, cmax + 1, -1, 0});
  return start;
}

// Steps of the pruned VTV program V T V ... T V: M = number of T actions, or
// -1 if the program has another shape.
int vtv_m(const DevView& d) {
  if (d.nact < 3 || (d.nact & 1) == 0) return -1;
  for (int a = 0; a < d.nact; ++a)
    if (sop::prog_op(d.hprog[a]) != ((a & 1) ? sop::OP_T : sop::OP_V)) return -1;
  return (d.nact - 1) / 2;
}

std::string dtype_name(bool f64) { return f64 ? "c128" : "c64"; }

// ---- tuning cache: a flat JSON object of string pairs
std::map<std::string, std::string> read_cache(const std::string& path) {
  std::map<std::string, std::string> m;
  std::ifstream f(path);
  if (!f) return m;
  std::stringstream ss;
  ss << f.rdbuf();
  const std::string s = ss.str();
  std::vector<std::string> strs;
  for (size_t i = 0; i < s.size(); ++i) {
    if (s[i] != '"') continue;
    const size_t j = s.find('"', i + 1);
    if (j == std::string::npos) break;
    strs.push_back(s.substr(i + 1, j - i - 1));
    i = j;
  }
  for (size_t k = 0; k + 1 < strs.size(); k += 2) m[strs[k]] = strs[k + 1];
  return m;
}

void write_cache(const std::string& path, const std::map<std::string, std::string>& m) {
  const std::string tmp = path + ".tmp";
  {
    std::ofstream f(tmp);
    if (!f) return;
    f << "{\n";
    size_t i = 0;
    for (const auto& kv : m) {
      f << "  \"" << kv.first << "\": \"" << kv.second << "\"" << (++i < m.size() ? "," : "")
        << "\n";
    }
    f << "}\n";
  }
  (void)std::rename(tmp.c_str(), path.c_str());
}

// Best (minimum) time of `reps` launches of fn on `st`, after one warm-up.
template <class F>
hipError_t time_min(hipStream_t st, int reps, F&& fn, double* ms_out) {
  hipEvent_t a, b;
  hipError_t e = hipEventCreate(&a);
  if (e != hipSuccess) return e;
  if ((e = hipEventCreate(&b)) != hipSuccess) {
    (void)hipEventDestroy(a);
    return e;
  }
  double best = 1e300;
  e = fn();
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  for (int r = 0; r < reps && e == hipSuccess; ++r) {
    if ((e = hipEventRecord(a, st)) != hipSuccess) break;
    if ((e = fn()) != hipSuccess) break;
    if ((e = hipEventRecord(b, st)) != hipSuccess) break;
    if ((e = hipEventSynchronize(b)) != hipSuccess) break;
    float ms = 0;
    if ((e = hipEventElapsedTime(&ms, a, b)) != hipSuccess) break;
    best = std::min(best, (double)ms);
  }
  (void)hipEventDestroy(a);
  (void)hipEventDestroy(b);
  *ms_out = best;
  return e;
}

}  // namespace

struct sop_batch {
  hipStream_t stream = nullptr;
  std::vector<sop_plan*> plans;
  std::vector<const DevView*> views;
  std::vector<Family1> fams;
  std::vector<Group3> groups;
  std::vector<int> solo;
  hipStream_t capture = nullptr;
  std::vector<hipStream_t> branches;
  hipEvent_t fork = nullptr;
  std::vector<hipEvent_t> joins;
  bool use_graphs = true;
  bool use_plane = true;
  bool use_queue = false;            // 3D groups as one work-queue launch
  long long spin_limit = 1LL << 21;  // polls of one queue wait
  hipGraphExec_t exec = nullptr;
  int64_t graph_nodes = 0;
  bool last_graph = false;
  // key of the captured graph
  std::vector<void*> key_psi;
  std::vector<int64_t> key_n;
  int key_conj = -1;
  bool key_valid = false;

  ~sop_batch() {
    if (exec) (void)hipGraphExecDestroy(exec);
    for (auto& f : fams)
      if (f.d_mem) (void)hipFree(f.d_mem);
    for (auto& g : groups) {
      if (g.d_mem) (void)hipFree(g.d_mem);
      if (g.d_rounds) (void)hipFree(g.d_rounds);
      if (g.d_ctrl) (void)hipFree(g.d_ctrl);
    }
    for (hipStream_t s : branches) (void)hipStreamDestroy(s);
    if (capture) (void)hipStreamDestroy(capture);
    if (fork) (void)hipEventDestroy(fork);
    for (hipEvent_t e : joins) (void)hipEventDestroy(e);
  }
};

namespace {

// ---- tuning of one 1D family on scratch states
sop_status tune_family(sop_batch* b, Family1& f) {
  const int nv = sop::k1b_variants(f.n, f.S);
  if (nv <= 1) return SOP_OK;
  const int cnt = std::min<int>((int)f.members.size(), 64);
  const size_t csize = f.f64 ? 16 : 8;
  const size_t one = (size_t)f.S * f.n * csize;
  void* scratch = nullptr;
  BMember1* d_mem = nullptr;
  if (hipMalloc(&scratch, one * cnt) != hipSuccess ||
      hipMalloc((void**)&d_mem, sizeof(BMember1) * cnt) != hipSuccess) {
    (void)hipGetLastError();
    if (scratch) (void)hipFree(scratch);
    return fail(SOP_ERR_NOMEM, "device allocation failed for batch tuning");
  }
  std::vector<BMember1> h(cnt);
  for (int i = 0; i < cnt; ++i) {
    const DevView& d = *b->views[f.members[i]];
    h[i].psi = (char*)scratch + one * i;
    h[i].vexp = d.vexp;
    h[i].kin = d.kin;
    h[i].tw = d.tw[0];
    h[i].prog = d.prog;
    h[i].nact = d.nact;
    h[i].nsteps = std::max(1, 64 / d.nact);
    h[i].conj = 0;
  }
  hipError_t e = hipMemsetAsync(scratch, 0, one * cnt, b->stream);
  if (e == hipSuccess)
    e = hipMemcpyAsync(d_mem, h.data(), sizeof(BMember1) * cnt, hipMemcpyHostToDevice,
                       b->stream);
  f.tuned_ms.assign(nv, -1.0);
  for (int v = 0; v < nv && e == hipSuccess; ++v) {
    double ms = 0;
    e = time_min(b->stream, 3, [&] { return sop::k1b_launch(f.n, f.S, f.f64, v, d_mem, cnt,
                                                            b->stream); }, &ms);
    if (e == hipSuccess) f.tuned_ms[v] = ms;
  }
  (void)hipStreamSynchronize(b->stream);
  (void)hipFree(scratch);
  (void)hipFree(d_mem);
  if (e != hipSuccess) return fail(SOP_ERR_HIP, std::string("batch tuning: ") + hipGetErrorString(e));
  f.variant = 0;
  for (int v = 1; v < nv; ++v)
    if (f.tuned_ms[v] < f.tuned_ms[f.variant]) f.variant = v;
  return SOP_OK;
}

// ---- tuning of one 3D lockstep group: each pass kind separately
sop_status tune_group(sop_batch* b, Group3& g) {
  const int cnt = std::min<int>((int)g.members.size(), 16);
  const size_t csize = g.f64 ? 16 : 8;
  const size_t one = (size_t)g.S * g.n * g.n * g.n * csize;
  void* scratch = nullptr;
  BMember3* d_mem = nullptr;
  if (hipMalloc(&scratch, one * cnt) != hipSuccess ||
      hipMalloc((void**)&d_mem, sizeof(BMember3) * cnt) != hipSuccess) {
    (void)hipGetLastError();
    if (scratch) (void)hipFree(scratch);
    return fail(SOP_ERR_NOMEM, "device allocation failed for batch tuning");
  }
  std::vector<BMember3> h(cnt);
  for (int i = 0; i < cnt; ++i) {
    const DevView& d = *b->views[g.members[i]];
    BMember3& m = h[i];
    std::memset(&m, 0, sizeof(m));
    m.psi = (char*)scratch + one * i;
    m.vexp = d.vexp;
    m.vtaus = d.vtaus;
    m.kin = d.kin;
    m.tw = d.tw[0];
    m.prog = d.prog;
    m.M = vtv_m(d);
    m.cycles = (int64_t)1 << 40;  // never the closing pass
    m.conj = 0;
    m.kin_stride = d.kin_stride;
  }
  hipError_t e = hipMemsetAsync(scratch, 0, one * cnt, b->stream);
  if (e == hipSuccess)
    e = hipMemcpyAsync(d_mem, h.data(), sizeof(BMember3) * cnt, hipMemcpyHostToDevice,
                       b->stream);
  auto pick = [&](int kind, std::vector<double>& ms, int* best) {
    const int nv = sop::k3b_variants(kind, g.n, g.f64);
    ms.assign(nv, -1.0);
    *best = 0;
    for (int v = 0; v < nv && e == hipSuccess; ++v) {
      if (sop::k3b_variant_width(kind, g.n, g.f64, v) == 0) continue;
      double t = 0;
      e = time_min(b->stream, 3, [&] {
        return sop::k3b_launch(kind, g.n, g.S, g.f64, v, d_mem, cnt, 1, b->stream);
      }, &t);
      if (e != hipSuccess) break;
      ms[v] = t;
      if (ms[*best] < 0 || t < ms[*best]) *best = v;
    }
  };
  pick(sop::B3_Z, g.ms_z, &g.vz);
  pick(sop::B3_Y, g.ms_y, &g.vy);
  pick(sop::B3_X, g.ms_x, &g.vx);
  (void)hipStreamSynchronize(b->stream);
  (void)hipFree(scratch);
  (void)hipFree(d_mem);
  if (e != hipSuccess) return fail(SOP_ERR_HIP, std::string("batch tuning: ") + hipGetErrorString(e));
  return SOP_OK;
}

std::string fam_key(const Family1& f) {
  return "1d/n" + std::to_string(f.n) + "/s" + std::to_string(f.S) + "/" + dtype_name(f.f64);
}
std::string grp_key(const Group3& g) {
  return "3d/n" + std::to_string(g.n) + "/s" + std::to_string(g.S) + "/" + dtype_name(g.f64);
}

// ---- enqueueing of one propagate call on the branch streams
hipError_t enqueue(sop_batch* b, const std::vector<int64_t>& nsteps, void* const* psi, int conj) {
  size_t br = 0;
  auto next = [&]() { return b->branches[br++ % b->branches.size()]; };
  for (Family1& f : b->fams) {
    bool any = false;
    for (int m : f.members) any = any || nsteps[m] > 0;
    if (!any) continue;
    hipError_t e = sop::k1b_launch(f.n, f.S, f.f64, f.variant, f.d_mem, (int)f.members.size(),
                                   next());
    if (e != hipSuccess) return e;
  }
  // lockstep chains: [lo, hi) of a group's members, the stream, and the
  // members still running at the current cycle (z-pass, y/x passes)
  struct Chain {
    const Group3* g;
    int lo, hi;
    hipStream_t st;
    int nz = hi - lo, nyx = hi - lo;
  };
  std::vector<Chain> chains;
  for (Group3& g : b->groups) {
    if (b->use_queue) {
      if (g.tickets <= 0) continue;
      hipError_t e = sop::k3q_launch(g.n, g.S, g.f64, g.d_mem, (int)g.members.size(),
                                     g.d_rounds, (int)g.nrounds, g.tickets, g.d_ctrl,
                                     b->spin_limit, next());
      if (e != hipSuccess) return e;
      continue;
    }
    for (const auto& ch : g.chains) chains.push_back({&g, ch.first, ch.second, next()});
  }
  // Every chain's cycle c is enqueued before any chain's cycle c + 1, so that
  // the chains start together when the launches are enqueued eagerly (a long
  // chain enqueued after all the others would start late); each chain keeps
  // its own stream, so the order of its own launches is unchanged.
  int64_t cmax = -1;
  for (const Chain& ch : chains) cmax = std::max(cmax, ch.g->cycles[ch.lo]);
  for (int64_t c = 0; c <= cmax; ++c) {
    for (Chain& ch : chains) {
      const Group3& g = *ch.g;
      const int64_t maxc = g.cycles[ch.lo];
      if (c > maxc) continue;
      BMember3* mem = g.d_mem + ch.lo;
      while (ch.nz > 0 && g.cycles[ch.lo + ch.nz - 1] < c) --ch.nz;
      while (ch.nyx > 0 && g.cycles[ch.lo + ch.nyx - 1] <= c) --ch.nyx;
      hipError_t e = sop::k3b_launch(sop::B3_Z, g.n, g.S, g.f64, g.vz, mem, ch.nz, c, ch.st);
      if (e != hipSuccess) return e;
      if (c == maxc) continue;
      if (b->use_plane && sop::k3b_plane(g.n, g.f64)) {
        if ((e = sop::k3b_launch(sop::B3_XY, g.n, g.S, g.f64, 0, mem, ch.nyx, c, ch.st)) !=
            hipSuccess)
          return e;
        continue;
      }
      if ((e = sop::k3b_launch(sop::B3_Y, g.n, g.S, g.f64, g.vy, mem, ch.nyx, c, ch.st)) !=
          hipSuccess)
        return e;
      if ((e = sop::k3b_launch(sop::B3_X, g.n, g.S, g.f64, g.vx, mem, ch.nyx, c, ch.st)) !=
          hipSuccess)
        return e;
    }
  }
  for (int m : b->solo) {
    if (nsteps[m] <= 0) continue;
    DevView d = *b->views[m];
    d.stream = next();
    d.graphs = nullptr;
    d.timer = nullptr;
    d.count = 1;
    hipError_t e = d.ndim == 1 ? sop::k1d_propagate(d, psi[m], nsteps[m], conj)
                               : sop::k3d_propagate(d, psi[m], nsteps[m], conj);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

// fork from `origin`, enqueue on the branches, join back into `origin`
hipError_t fork_join(sop_batch* b, hipStream_t origin, const std::vector<int64_t>& nsteps,
                     void* const* psi, int conj) {
  hipError_t e = hipEventRecord(b->fork, origin);
  if (e != hipSuccess) return e;
  for (hipStream_t s : b->branches)
    if ((e = hipStreamWaitEvent(s, b->fork, 0)) != hipSuccess) return e;
  if ((e = enqueue(b, nsteps, psi, conj)) != hipSuccess) return e;
  for (size_t i = 0; i < b->branches.size(); ++i) {
    if ((e = hipEventRecord(b->joins[i], b->branches[i])) != hipSuccess) return e;
    if ((e = hipStreamWaitEvent(origin, b->joins[i], 0)) != hipSuccess) return e;
  }
  return hipSuccess;
}

int64_t count_nodes(const sop_batch* b, const std::vector<int64_t>& nsteps) {
  int64_t n = (int64_t)b->fams.size();
  for (const Group3& g : b->groups) {
    if (b->use_queue) {
      n += 2;
      continue;
    }
    const int per = (b->use_plane && sop::k3b_plane(g.n, g.f64)) ? 2 : 3;
    for (const auto& ch : g.chains) n += per * g.cycles[ch.first] + 1;
  }
  for (int m : b->solo) {
    const DevView& d = *b->views[m];
    n += d.ndim == 1 ? 1 : 3 * (int64_t)d.nact * nsteps[m] + 1;
  }
  return n;
}

}  // namespace

extern "C" {

sop_status sop_batch_create(sop_plan* const* plans, int count, void* hip_stream,
                            sop_batch** out) {
  if (!plans || !out) return fail(SOP_ERR_INVALID, "NULL argument");
  if (count < 1 || count > 65535) return fail(SOP_ERR_INVALID, "count must be 1..65535");
  for (int i = 0; i < count; ++i)
    if (!plans[i]) return fail(SOP_ERR_INVALID, "plan " + std::to_string(i) + " is NULL");
  sop_batch* b = new (std::nothrow) sop_batch();
  if (!b) return fail(SOP_ERR_NOMEM, "host allocation failed");
  struct Guard {
    sop_batch* b;
    bool keep = false;
    ~Guard() {
      if (!keep) delete b;
    }
  } guard{b};
  b->stream = (hipStream_t)hip_stream;
  b->plans.assign(plans, plans + count);
  for (int i = 0; i < count; ++i) b->views.push_back(sop::plan_view(plans[i]));

  // grouping
  std::map<std::string, int> fidx, gidx;
  for (int i = 0; i < count; ++i) {
    const DevView& d = *b->views[i];
    if (d.ndim == 1) {
      const std::string k = std::to_string(d.n[0]) + "/" + std::to_string(d.S) + "/" +
                            dtype_name(d.f64);
      auto it = fidx.find(k);
      if (it == fidx.end()) {
        Family1 f;
        f.n = d.n[0];
        f.S = d.S;
        f.f64 = d.f64;
        it = fidx.emplace(k, (int)b->fams.size()).first;
        b->fams.push_back(f);
      }
      b->fams[it->second].members.push_back(i);
    } else if (sop::k3b_supported(d.n[0], d.S) && vtv_m(d) > 0 &&
               d.eig == sop::eig_form(3, d.S)) {
      const std::string k = std::to_string(d.n[0]) + "/" + std::to_string(d.S) + "/" +
                            dtype_name(d.f64);
      auto it = gidx.find(k);
      if (it == gidx.end()) {
        Group3 g;
        g.n = d.n[0];
        g.S = d.S;
        g.f64 = d.f64;
        it = gidx.emplace(k, (int)b->groups.size()).first;
        b->groups.push_back(g);
      }
      b->groups[it->second].members.push_back(i);
    } else {
      b->solo.push_back(i);
    }
  }
  for (Family1& f : b->fams)
    if (hipMalloc((void**)&f.d_mem, sizeof(BMember1) * f.members.size()) != hipSuccess) {
      (void)hipGetLastError();
      return fail(SOP_ERR_NOMEM, "device allocation failed for batch descriptors");
    }
  for (Group3& g : b->groups) {
    const size_t cb = sop::q_ctrl_words((int)g.members.size()) * sizeof(unsigned long long);
    if (hipMalloc((void**)&g.d_mem, sizeof(BMember3) * g.members.size()) != hipSuccess ||
        hipMalloc((void**)&g.d_ctrl, cb) != hipSuccess) {
      (void)hipGetLastError();
      return fail(SOP_ERR_NOMEM, "device allocation failed for batch descriptors");
    }
    HIPTRY(hipMemset(g.d_ctrl, 0, cb));
  }

  // persistent grid sizes of the work-queue launches (an occupancy query,
  // made here rather than while a propagate call is being captured)
  for (const Group3& g : b->groups) (void)sop::k3q_grid(g.n, g.S, g.f64);

  // streams and events
  const int nbranch = std::max<int>(
      1, std::min<int>(kMaxBranches,
                       (int)(b->fams.size() + 6 * b->groups.size() + b->solo.size())));
  HIPTRY(hipStreamCreateWithFlags(&b->capture, hipStreamNonBlocking));
  for (int i = 0; i < nbranch; ++i) {
    hipStream_t s;
    HIPTRY(hipStreamCreateWithFlags(&s, hipStreamNonBlocking));
    b->branches.push_back(s);
    hipEvent_t e;
    HIPTRY(hipEventCreateWithFlags(&e, hipEventDisableTiming));
    b->joins.push_back(e);
  }
  HIPTRY(hipEventCreateWithFlags(&b->fork, hipEventDisableTiming));

  // tuning
  const char* tune_env = std::getenv("SOPROP_TUNE");
  const bool tune = !(tune_env && std::strcmp(tune_env, "0") == 0);
  const char* cache_env = std::getenv("SOPROP_TUNE_CACHE");
  std::map<std::string, std::string> cache;
  if (cache_env && *cache_env) cache = read_cache(cache_env);
  bool cache_dirty = false;
  auto cached = [&](const std::string& k, int nv, int* v) {
    auto it = cache.find(k);
    if (it == cache.end()) return false;
    const int x = std::atoi(it->second.c_str());
    if (x < 0 || x >= nv) return false;
    *v = x;
    return true;
  };
  for (Family1& f : b->fams) {
    const int nv = sop::k1b_variants(f.n, f.S);
    if (cached(fam_key(f), nv, &f.variant)) {
      f.from_cache = true;
      continue;
    }
    if (!tune) continue;
    sop_status st = tune_family(b, f);
    if (st != SOP_OK) return st;
    if (nv > 1) {
      cache[fam_key(f)] = std::to_string(f.variant);
      cache_dirty = true;
    }
  }
  for (Group3& g : b->groups) {
    const std::string k = grp_key(g);
    auto ok = [&](int kind, int v) { return sop::k3b_variant_width(kind, g.n, g.f64, v) > 0; };
    int vz, vy, vx;
    if (cached(k + "/z", 2, &vz) && cached(k + "/y", 3, &vy) && cached(k + "/x", 3, &vx) &&
        ok(sop::B3_Z, vz) && ok(sop::B3_Y, vy) && ok(sop::B3_X, vx)) {
      g.vz = vz;
      g.vy = vy;
      g.vx = vx;
      g.from_cache = true;
      continue;
    }
    if (!tune) continue;
    sop_status st = tune_group(b, g);
    if (st != SOP_OK) return st;
    cache[k + "/z"] = std::to_string(g.vz);
    cache[k + "/y"] = std::to_string(g.vy);
    cache[k + "/x"] = std::to_string(g.vx);
    cache_dirty = true;
  }
  if (cache_dirty && cache_env && *cache_env) write_cache(cache_env, cache);
  HIPTRY(hipStreamSynchronize(b->stream));
  guard.keep = true;
  *out = b;
  return SOP_OK;
}

sop_status sop_batch_destroy(sop_batch* b) {
  if (b) {
    (void)hipStreamSynchronize(b->stream);
    for (hipStream_t s : b->branches) (void)hipStreamSynchronize(s);
    delete b;
  }
  return SOP_OK;
}

sop_status sop_batch_propagate(sop_batch* b, void* const* psi, const int64_t* nsteps,
                               int direction) {
  if (!b || !psi || !nsteps) return fail(SOP_ERR_INVALID, "NULL argument");
  if (direction != 1 && direction != -1) return fail(SOP_ERR_INVALID, "direction must be +1 or -1");
  const int count = (int)b->plans.size();
  for (int i = 0; i < count; ++i) {
    if (!psi[i]) return fail(SOP_ERR_INVALID, "psi " + std::to_string(i) + " is NULL");
    if (nsteps[i] < 0) return fail(SOP_ERR_INVALID, "nsteps must be >= 0");
  }
  const int conj = direction < 0 ? 1 : 0;
  std::vector<int64_t> ns(nsteps, nsteps + count);
  const bool same = b->key_valid && b->key_conj == conj && b->key_n == ns &&
                    std::equal(b->key_psi.begin(), b->key_psi.end(), psi);
  if (same && b->exec) {
    HIPTRY(hipGraphLaunch(b->exec, b->stream));
    return SOP_OK;
  }
  if (!same) {
    // new descriptors: wait until no earlier launch reads the old ones
    HIPTRY(hipStreamSynchronize(b->stream));
    if (b->exec) {
      (void)hipGraphExecDestroy(b->exec);
      b->exec = nullptr;
    }
    for (Family1& f : b->fams) {
      std::vector<int> order = f.members;
      std::stable_sort(order.begin(), order.end(), [&](int x, int y) {
        return ns[x] * b->views[x]->nact > ns[y] * b->views[y]->nact;
      });
      std::vector<BMember1> h(order.size());
      for (size_t i = 0; i < order.size(); ++i) {
        const DevView& d = *b->views[order[i]];
        h[i].psi = psi[order[i]];
        h[i].vexp = d.vexp;
        h[i].kin = d.kin;
        h[i].tw = d.tw[0];
        h[i].prog = d.prog;
        h[i].nact = d.nact;
        h[i].nsteps = ns[order[i]];
        h[i].conj = conj;
      }
      HIPTRY(hipMemcpy(f.d_mem, h.data(), sizeof(BMember1) * h.size(), hipMemcpyHostToDevice));
    }
    for (Group3& g : b->groups) {
      std::vector<int> order = g.members;
      std::stable_sort(order.begin(), order.end(), [&](int x, int y) {
        return (int64_t)vtv_m(*b->views[x]) * ns[x] > (int64_t)vtv_m(*b->views[y]) * ns[y];
      });
      std::vector<BMember3> h(order.size());
      g.max_cycles = 0;
      g.cycles.assign(order.size(), 0);
      g.chains.clear();
      for (size_t i = 0; i < order.size(); ++i) {
        const int mi = order[i];
        const DevView& d = *b->views[mi];
        BMember3& m = h[i];
        std::memset(&m, 0, sizeof(m));
        m.psi = psi[mi];
        m.vexp = d.vexp;
        m.vtaus = d.vtaus;
        m.kin = d.kin;
        m.tw = d.tw[0];
        m.prog = d.prog;
        m.M = vtv_m(d);
        m.cycles = (int64_t)m.M * ns[mi];
        m.conj = conj;
        m.kin_stride = d.kin_stride;
        g.max_cycles = std::max(g.max_cycles, m.cycles);
        g.cycles[i] = m.cycles;
        if (m.cycles > 0 && (g.chains.empty() || 4 * m.cycles < g.cycles[g.chains.back().first]))
          g.chains.push_back({(int)i, (int)i + 1});
        else if (m.cycles > 0)
          g.chains.back().second = (int)i + 1;
      }
      HIPTRY(hipMemcpy(g.d_mem, h.data(), sizeof(BMember3) * h.size(), hipMemcpyHostToDevice));
      std::vector<sop::QRound> rounds;
      g.tickets = build_rounds(g.cycles, sop::k3q_tiles(sop::B3_Z, g.n, g.S, g.f64),
                               sop::k3q_tiles(sop::B3_Y, g.n, g.S, g.f64), rounds);
      g.nrounds = (int64_t)rounds.size() - 1;
      if (rounds.size() > g.rounds_cap) {
        if (g.d_rounds) (void)hipFree(g.d_rounds);
        g.d_rounds = nullptr;
        g.rounds_cap = 0;
        if (hipMalloc((void**)&g.d_rounds, rounds.size() * sizeof(sop::QRound)) != hipSuccess) {
          (void)hipGetLastError();
          b->key_valid = false;
          return fail(SOP_ERR_NOMEM, "device allocation failed for the work-queue rounds");
        }
        g.rounds_cap = rounds.size();
      }
      HIPTRY(hipMemcpy(g.d_rounds, rounds.data(), rounds.size() * sizeof(sop::QRound),
                       hipMemcpyHostToDevice));
    }
    b->key_psi.assign(psi, psi + count);
    b->key_n = ns;
    b->key_conj = conj;
    b->key_valid = true;
  }
  b->graph_nodes = count_nodes(b, ns);
  if (!b->use_graphs || b->graph_nodes > kGraphNodeCap) {
    b->last_graph = false;
    HIPTRY(fork_join(b, b->stream, ns, psi, conj));
    return SOP_OK;
  }
  HIPTRY(hipStreamBeginCapture(b->capture, hipStreamCaptureModeThreadLocal));
  hipError_t le = fork_join(b, b->capture, ns, psi, conj);
  hipGraph_t graph = nullptr;
  hipError_t ce = hipStreamEndCapture(b->capture, &graph);
  if (le != hipSuccess || ce != hipSuccess) {
    if (graph) (void)hipGraphDestroy(graph);
    b->key_valid = false;
    return fail(SOP_ERR_HIP, std::string("batch capture: ") +
                                 hipGetErrorString(le != hipSuccess ? le : ce));
  }
  hipGraphExec_t x = nullptr;
  hipError_t ie = hipGraphInstantiate(&x, graph, nullptr, nullptr, 0);
  (void)hipGraphDestroy(graph);
  if (ie != hipSuccess) {
    b->key_valid = false;
    return fail(SOP_ERR_HIP, std::string("batch graph instantiation: ") + hipGetErrorString(ie));
  }
  b->exec = x;
  b->last_graph = true;
  HIPTRY(hipGraphLaunch(b->exec, b->stream));
  return SOP_OK;
}

sop_status sop_batch_set_option(sop_batch* b, int option, int value) {
  if (!b) return fail(SOP_ERR_INVALID, "batch is NULL");
  if (option != SOP_OPT_GRAPHS && option != SOP_OPT_PLANE_PASS && option != SOP_OPT_QUEUE &&
      option != SOP_OPT_QUEUE_SPIN)
    return fail(SOP_ERR_INVALID, "unknown option");
  if (option == SOP_OPT_QUEUE_SPIN && value < 1)
    return fail(SOP_ERR_INVALID, "the queue's poll limit must be >= 1");
  HIPTRY(hipStreamSynchronize(b->stream));
  if (option == SOP_OPT_GRAPHS)
    b->use_graphs = value != 0;
  else if (option == SOP_OPT_PLANE_PASS)
    b->use_plane = value != 0;
  else if (option == SOP_OPT_QUEUE)
    b->use_queue = value != 0;
  else
    b->spin_limit = value;
  if (b->exec) {
    (void)hipGraphExecDestroy(b->exec);
    b->exec = nullptr;
  }
  return SOP_OK;
}

sop_status sop_batch_check(sop_batch* b) {
  if (!b) return fail(SOP_ERR_INVALID, "batch is NULL");
  HIPTRY(hipStreamSynchronize(b->stream));
  int aborted = 0;
  for (Group3& g : b->groups) {
    unsigned long long flag = 0;
    HIPTRY(hipMemcpy(&flag, g.d_ctrl + 2 * sop::kQSlot, sizeof(flag), hipMemcpyDeviceToHost));
    if (flag != 0) {
      ++aborted;
      const unsigned long long zero = 0;
      HIPTRY(hipMemcpy(g.d_ctrl + 2 * sop::kQSlot, &zero, sizeof(zero), hipMemcpyHostToDevice));
    }
  }
  if (aborted > 0)
    return fail(SOP_ERR_STATE, std::to_string(aborted) +
                                   " work-queue launch(es) ran a wait out of polls and left "
                                   "their members unfinished");
  return SOP_OK;
}

sop_status sop_batch_describe(const sop_batch* b, char* buf, size_t len, size_t* needed) {
  if (!b) return fail(SOP_ERR_INVALID, "batch is NULL");
  std::ostringstream o;
  auto arr = [&](const std::vector<double>& v) {
    o << "[";
    for (size_t i = 0; i < v.size(); ++i) {
      if (i) o << ", ";
      if (v[i] < 0)
        o << "null";
      else
        o << v[i];
    }
    o << "]";
  };
  auto members = [&](const std::vector<int>& v) {
    o << "[";
    for (size_t i = 0; i < v.size(); ++i) o << (i ? ", " : "") << v[i];
    o << "]";
  };
  o << "{\"families\": [";
  for (size_t i = 0; i < b->fams.size(); ++i) {
    const Family1& f = b->fams[i];
    o << (i ? ", " : "") << "{\"n\": " << f.n << ", \"S\": " << f.S << ", \"dtype\": \""
      << dtype_name(f.f64) << "\", \"members\": ";
    members(f.members);
    o << ", \"variant\": " << f.variant << ", \"schedule\": \""
      << sop::k1b_variant_name(f.n, f.S, f.variant, f.f64) << "\", \"from_cache\": "
      << (f.from_cache ? "true" : "false") << ", \"tuned_ms\": ";
    arr(f.tuned_ms);
    o << "}";
  }
  o << "], \"groups\": [";
  for (size_t i = 0; i < b->groups.size(); ++i) {
    const Group3& g = b->groups[i];
    o << (i ? ", " : "") << "{\"n\": " << g.n << ", \"S\": " << g.S << ", \"dtype\": \""
      << dtype_name(g.f64) << "\", \"members\": ";
    members(g.members);
    o << ", \"z_cols\": " << sop::k3b_variant_width(sop::B3_Z, g.n, g.f64, g.vz)
      << ", \"y_cols\": " << sop::k3b_variant_width(sop::B3_Y, g.n, g.f64, g.vy)
      << ", \"x_rows\": " << sop::k3b_variant_width(sop::B3_X, g.n, g.f64, g.vx)
      << ", \"plane\": "
      << ((!b->use_queue && b->use_plane && sop::k3b_plane(g.n, g.f64)) ? "true" : "false")
      << ", \"queue\": " << (b->use_queue ? "true" : "false") << ", \"rounds\": " << g.nrounds
      << ", \"tickets\": " << g.tickets << ", \"queue_grid\": "
      << sop::k3q_grid(g.n, g.S, g.f64)
      << ", \"from_cache\": " << (g.from_cache ? "true" : "false") << ", \"tuned_ms\": {\"z\": ";
    arr(g.ms_z);
    o << ", \"y\": ";
    arr(g.ms_y);
    o << ", \"x\": ";
    arr(g.ms_x);
    o << "}, \"max_cycles\": " << g.max_cycles << ", \"chains\": [";
    for (size_t c = 0; c < g.chains.size(); ++c)
      o << (c ? ", " : "") << "[" << g.chains[c].second - g.chains[c].first << ", "
        << g.cycles[g.chains[c].first] << "]";
    o << "]}";
  }
  o << "], \"solo\": ";
  members(b->solo);
  o << ", \"branches\": " << b->branches.size() << ", \"graph\": "
    << (b->last_graph ? "true" : "false") << ", \"graph_nodes\": " << b->graph_nodes << "}";
  const std::string s = o.str();
  if (needed) *needed = s.size() + 1;
  if (buf && len > 0) {
    const size_t n = std::min(len - 1, s.size());
    std::memcpy(buf, s.data(), n);
    buf[n] = '\0';
  }
  return SOP_OK;
}

}  // extern "C"
