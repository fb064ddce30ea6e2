// batch.cpp -- host side of the batched engine: validation, descriptor tables,
// lane groups and team layout of the team sweep, workspace, the per-chunk launch
// sequence (optionally captured once in a hipGraph and replayed), and the
// autotuner (team layout of the team sweep, row unroll of the per-lane sweep).
//
// A chunk of T iterations is: partitions of every active instance for the T
// iterations; then per iteration the shared block Grams, the per-lane block
// inverses, the per-lane sweeps and z/dual steps; then the KKT check, the
// penalty rule and the activity count.  The host reads one integer (active
// lanes) per chunk.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <new>
#include <string>
#include <utility>
#include <vector>

#include "rac_internal.h"
#include "racmb.h"

using namespace rac;

namespace {

#define BCHK(expr)                                   \
  do {                                               \
    hipError_t e_ = (expr);                          \
    if (e_ != hipSuccess) return RAC_ERR_DEVICE;     \
  } while (0)

struct DevBufs {
  std::vector<void*> owned;
  template <typename T> bool alloc(T** p, size_t count) {
    void* q = nullptr;
    if (count == 0) count = 1;
    if (hipMalloc(&q, sizeof(T) * count) != hipSuccess) return false;
    owned.push_back(q);
    *p = (T*)q;
    return true;
  }
  void release() {
    for (void* q : owned) (void)hipFree(q);
    owned.clear();
  }
};

DevScalars fresh(double beta) {
  DevScalars s{};
  s.beta = beta;
  s.kkt = NAN;
  s.kkt_prev = -1.0;
  s.rp_first = -1.0;
  s.objective = NAN;
  s.fail_key = ~0ULL;
  return s;
}

std::string tune_cache_path() {
  const char* p = std::getenv("RACMB_TUNE_CACHE");
  if (p && *p) return p;
  const char* home = std::getenv("HOME");
  return std::string(home ? home : "/tmp") + "/.cache/racmb_tune.txt";
}

}  // namespace

struct rac_batch_s {
  rac_batch_opts O{};
  int ninst = 0, nunits = 0, SP = 16, T = 1;
  std::vector<BInst> hinst;
  std::vector<BUnit> hunit;
  std::vector<int64_t> unit_n;
  DevBufs buf;
  BatchArgs A{};
  BInst* dinst = nullptr;
  BUnit* dunit = nullptr;
  int2* gtasks = nullptr;
  int ngt = 0;
  int nslot = 1;               // Gram / inverse slots: one per iteration of a chunk, or one
  int32_t host_active = 0;
  int64_t k = 0;
  hipStream_t cs = nullptr;           // the batch's own stream (capturable)
  hipEvent_t ev = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t gexec = nullptr;
  bool graph_used = false;
  std::string tune_key;
  // team sweep: lane groups, their LPT costs, and the current team layout
  bool team = false;
  TeamArgs TA{};
  std::vector<TGroup> hgroups;
  std::vector<double> gcost;   // predicted cost of a group (LPT key)
  std::vector<int> gwidth;     // team width a group runs on (1: solo, 16 or 32)
  // the two width sets: with solo groups (chosen at creation) and teams only, and the
  // predicted cost of each group under each; solo_on: the first set is in use
  std::vector<int> gw_solo, gw_team;
  std::vector<double> gc_solo, gc_team;
  bool solo_on = false;
  int lay0_k32 = 0, lay0_k16 = 0, lay0_ks = 0;   // layout of the solo set (tuned at creation)
  int32_t decided_active = -1;                   // active lanes when the widths were last decided
  int max_teams = 0;           // teams of the widest split: one per resident workgroup
  int resident = 0;            // team-sweep workgroups resident at once (the launch size)
  int k32 = 0, k16 = 0, ks = 0;   // current layout: teams of 32 and 16 workgroups, solo workers
  int32_t* dteam_w = nullptr;
  int64_t* dteam_part = nullptr;
  int32_t* dblk_team = nullptr;
  int32_t* dblk_member = nullptr;
  TGroup* dgroups = nullptr;
  int2* dkkt_tasks = nullptr;   // (group, pair of 64-column chunks) of the grouped KKT check
  int nkkt_tasks = 0;
  int32_t* dteam_off = nullptr;
  int32_t* dteam_list = nullptr;
  // per-phase timing (events around every launch; chunks are then launched directly)
  bool timing = false;
  std::vector<hipEvent_t> ev_t;
  std::vector<int> ev_phase;
  double phase_ms[RAC_NUM_PHASES] = {};
  int64_t phase_count[RAC_NUM_PHASES] = {};
};

namespace {

// Events around one launch when timing is on (never inside a graph capture).
struct BTimer {
  rac_batch b;
  hipStream_t st;
  hipError_t begin() {
    if (!b->timing) return hipSuccess;
    const size_t i = 2 * b->ev_phase.size();
    while (b->ev_t.size() < i + 2) {
      hipEvent_t e;
      hipError_t r = hipEventCreate(&e);
      if (r != hipSuccess) return r;
      b->ev_t.push_back(e);
    }
    return hipEventRecord(b->ev_t[i], st);
  }
  hipError_t end(int phase) {
    if (!b->timing) return hipSuccess;
    const size_t i = 2 * b->ev_phase.size();
    b->ev_phase.push_back(phase);
    return hipEventRecord(b->ev_t[i + 1], st);
  }
};

rac_status enqueue_chunk(rac_batch b, int Tc, hipStream_t st) {
  BatchArgs a = b->A;
  a.T = Tc;
  BTimer tm{b, st};
  BCHK(tm.begin());
  BCHK(launch_bperm(a, st));
  BCHK(tm.end(RAC_PHASE_PARTITION));
  // The Grams and inverses of an iteration depend only on its partition and on the
  // penalties, which change only at the check that ends a chunk: with a slot per
  // iteration they are formed for the whole chunk in one launch each (no launch tail
  // per iteration); otherwise at each iteration into the one slot.
  auto assemble = [&](int t0, int nt, int tk0) -> rac_status {
    BatchGramArgs g{a.dtype, b->O.precision, a.sp, b->ngt, t0, nt, a.gslot, a.inst, b->gtasks, a.perm,
                    a.inst_active, const_cast<double*>(a.G)};
    BCHK(tm.begin());
    BCHK(launch_bgram(g, st));
    BCHK(tm.end(RAC_PHASE_GRAM));
    BCHK(tm.begin());
    BCHK(launch_binv(a, t0, nt, tk0, st));
    BCHK(tm.end(RAC_PHASE_FACTOR));
    return RAC_OK;
  };
  const bool chunkwide = a.mslot != 0;
  if (chunkwide) {
    const rac_status e = assemble(0, Tc, 0);
    if (e != RAC_OK) return e;
  }
  for (int t = 0; t < Tc; ++t) {
    if (!chunkwide) {
      const rac_status e = assemble(t, 1, t);
      if (e != RAC_OK) return e;
    }
    BatchArgs at = a;                     // the sweep reads iteration t's inverses
    at.Minv = a.Minv + t * a.mslot;
    BCHK(tm.begin());
    if (b->team) BCHK(launch_tsweep(at, b->TA, t, st));
    else BCHK(launch_bsweep(at, t, st));
    BCHK(tm.end(RAC_PHASE_SWEEP));
    BCHK(tm.begin());
    BCHK(launch_bzdual(a, st));
    BCHK(tm.end(RAC_PHASE_ZDUAL));
  }
  BCHK(tm.begin());
  if (b->team) BCHK(launch_gkkt(a, b->dgroups, b->dkkt_tasks, b->nkkt_tasks, st));
  BCHK(launch_bcheck(a, Tc, Tc == b->T ? 1 : 0, b->team ? 1 : 0, st));
  BCHK(tm.end(RAC_PHASE_CHECK));
  return RAC_OK;
}

rac_status collect_timing(rac_batch b) {
  if (!b->timing) return RAC_OK;
  for (size_t q = 0; q < b->ev_phase.size(); ++q) {
    float ms = 0.f;
    BCHK(hipEventElapsedTime(&ms, b->ev_t[2 * q], b->ev_t[2 * q + 1]));
    b->phase_ms[b->ev_phase[q]] += ms;
    b->phase_count[b->ev_phase[q]] += 1;
  }
  b->ev_phase.clear();
  return RAC_OK;
}

// Snapshot / restore of the lane state around tuning trials.
struct Snapshot {
  std::vector<char> bytes;
};

// Bytes of the lane state: x, z, xi, z_prev and u of every lane, the lanes' device
// scalars, the iteration counter and the activity flags.
size_t state_bytes(const rac_batch b) {
  int64_t xs = 0, us = 0;
  for (const BUnit& u : b->hunit) { xs += u.n; us += u.rows; }
  return sizeof(double) * (4 * xs + us) + sizeof(DevScalars) * b->nunits + sizeof(int64_t) +
         sizeof(int32_t) * (b->ninst + 1);
}

// Copies the lane state to (save) or from host memory p (state_bytes(b) bytes).
rac_status state_xfer(rac_batch b, bool save, char* p) {
  int64_t xs = 0, us = 0;
  for (const BUnit& u : b->hunit) { xs += u.n; us += u.rows; }
  auto mv = [&](void* dev, size_t n) -> hipError_t {
    hipError_t e = save ? hipMemcpy(p, dev, n, hipMemcpyDeviceToHost) : hipMemcpy(dev, p, n, hipMemcpyHostToDevice);
    p += n;
    return e;
  };
  BCHK(mv(b->A.X, sizeof(double) * xs));
  BCHK(mv(b->A.Z, sizeof(double) * xs));
  BCHK(mv(b->A.XI, sizeof(double) * xs));
  BCHK(mv(b->A.ZP, sizeof(double) * xs));
  BCHK(mv(b->A.U, sizeof(double) * us));
  BCHK(mv(b->A.sc, sizeof(DevScalars) * b->nunits));
  BCHK(mv(b->A.kdev, sizeof(int64_t)));
  BCHK(mv(b->A.inst_active, sizeof(int32_t) * b->ninst));
  BCHK(mv(b->A.nactive, sizeof(int32_t)));
  return RAC_OK;
}

rac_status state_copy(rac_batch b, bool save, Snapshot& s) {
  if (save) s.bytes.resize(state_bytes(b));
  return state_xfer(b, save, s.bytes.data());
}

struct BatchStateHeader {
  uint64_t magic;
  int64_t nunits, ninst, state_bytes;
  int64_t k;                // iterations run by the batch
  int64_t scalars_bytes;
  int64_t solo_on;          // the lane groups' widths in use (solo groups or teams only)
};
constexpr uint64_t kBatchStateMagic = 0x5241434241544348ULL;   // "RACBATCH"

// Longest-processing-time assignment of the groups of one team width to k teams;
// returns the largest team load and fills lists.
double lpt(const rac_batch b, int width, int k, std::vector<std::vector<int32_t>>* lists) {
  if (lists) lists->assign(k, {});
  if (k <= 0) return 0.0;
  std::vector<int> order;
  for (int g = 0; g < (int)b->hgroups.size(); ++g)
    if (b->gwidth[g] == width) order.push_back(g);
  std::stable_sort(order.begin(), order.end(), [&](int x, int y) { return b->gcost[x] > b->gcost[y]; });
  std::vector<double> load(k, 0.0);
  for (int g : order) {
    int best = 0;
    for (int t = 1; t < k; ++t)
      if (load[t] < load[best]) best = t;
    load[best] += b->gcost[g];
    if (lists) (*lists)[best].push_back(g);
  }
  return *std::max_element(load.begin(), load.end());
}

// Team layout with k32 teams of 32 workgroups and k16 teams of 16 (a group runs
// on a team of its own width, so its arithmetic never depends on the layout and
// every layout gives bit-identical results).  Teams are placed inside one XCD
// each when the resident workgroups split evenly over the eight XCDs; the table
// gives every workgroup of the launch its team (or -1) and member index.  The
// epoch flags restart from zero, since a team may change its width.
rac_status set_team_layout(rac_batch b, int k32, int k16, int ks) {
  std::vector<std::vector<int32_t>> l32, l16, l1;
  lpt(b, 32, k32, &l32);
  lpt(b, 16, k16, &l16);
  lpt(b, 1, ks, &l1);
  const int nteams = k32 + k16 + ks;
  std::vector<int32_t> off(nteams + 1, 0), flat, tw(nteams);
  std::vector<int64_t> tpart(nteams);
  int64_t poff = 0;
  for (int t = 0; t < nteams; ++t) {
    const std::vector<int32_t>& L = t < k32 ? l32[t] : (t < k32 + k16 ? l16[t - k32] : l1[t - k32 - k16]);
    off[t] = (int32_t)flat.size();
    flat.insert(flat.end(), L.begin(), L.end());
    tw[t] = t < k32 ? 32 : (t < k32 + k16 ? 16 : 1);
    tpart[t] = poff;
    if (tw[t] > 1) poff += 2 * 1024 * (int64_t)tw[t];   // solo workers exchange nothing
  }
  off[nteams] = (int32_t)flat.size();
  const int R = b->resident;
  std::vector<int32_t> bt(R, -1), bm(R, 0);
  if (R % 8 == 0 && R / 8 >= 32) {
    const int per = R / 8;
    std::vector<int> used(8, 0);
    for (int t = 0; t < nteams; ++t) {       // widest first: teams of 32, of 16, then solo workers
      int x = 0;
      if (tw[t] == 1) {                      // solo workers go to the least used XCD
        for (int y = 1; y < 8; ++y)
          if (used[y] < used[x]) x = y;
        if (used[x] + 1 > per) x = 8;
      } else {
        while (x < 8 && used[x] + tw[t] > per) ++x;
      }
      if (x == 8) return RAC_ERR_ARG;        // cannot happen: the widths sum to at most R
      for (int m = 0; m < tw[t]; ++m) {
        const int blk = 8 * (used[x] + m) + x;
        bt[blk] = t;
        bm[blk] = m;
      }
      used[x] += tw[t];
    }
  } else {
    int next = 0;
    for (int t = 0; t < nteams; ++t)
      for (int m = 0; m < tw[t]; ++m, ++next) { bt[next] = t; bm[next] = m; }
  }
  BCHK(hipDeviceSynchronize());
  BCHK(hipMemcpy(b->dteam_off, off.data(), sizeof(int32_t) * off.size(), hipMemcpyHostToDevice));
  if (!flat.empty())
    BCHK(hipMemcpy(b->dteam_list, flat.data(), sizeof(int32_t) * flat.size(), hipMemcpyHostToDevice));
  BCHK(hipMemcpy(b->dteam_w, tw.data(), sizeof(int32_t) * nteams, hipMemcpyHostToDevice));
  BCHK(hipMemcpy(b->dteam_part, tpart.data(), sizeof(int64_t) * nteams, hipMemcpyHostToDevice));
  BCHK(hipMemcpy(b->dblk_team, bt.data(), sizeof(int32_t) * R, hipMemcpyHostToDevice));
  BCHK(hipMemcpy(b->dblk_member, bm.data(), sizeof(int32_t) * R, hipMemcpyHostToDevice));
  BCHK(hipMemset(b->TA.flags, 0, sizeof(uint32_t) * (size_t)b->max_teams * 128));
  BCHK(hipDeviceSynchronize());
  b->TA.nteams = nteams;
  b->TA.nblocks = R;
  b->k32 = k32;
  b->k16 = k16;
  b->ks = ks;
  if (b->gexec) {   // a captured graph holds the old launch configuration
    (void)hipGraphExecDestroy(b->gexec);
    (void)hipGraphDestroy(b->graph);
    b->gexec = nullptr;
    b->graph = nullptr;
  }
  return RAC_OK;
}

// Layouts worth trying, best predicted first: every split of the resident
// workgroups into teams of 32 and 16 that gives each width it needs a team,
// ranked by the largest predicted team load.
struct Layout {
  int k32, k16, ks;
  bool operator==(const Layout& o) const { return k32 == o.k32 && k16 == o.k16 && ks == o.ks; }
};

// A solo workgroup reads the block's columns as aligned 4-element vectors at clamped
// rows, so the quad that holds a column's last row may reach past it, up to the
// column's leading dimension: that needs ldF a multiple of 4, F aligned to 4 elements,
// and the last column's ldF elements inside F's device allocation.
static bool solo_layout_ok(const rac_problem& P) {
  const size_t esz = P.F_dtype == RAC_DT_F64 ? 8 : (P.F_dtype == RAC_DT_F32 ? 4 : 2);
  if (P.ldF % 4 != 0 || (uintptr_t)P.F % (4 * esz) != 0) return false;
  void* base = nullptr;
  size_t size = 0;
  if (hipMemGetAddressRange(&base, &size, const_cast<void*>(P.F)) != hipSuccess) {
    (void)hipGetLastError();
    return false;
  }
  return (uintptr_t)P.F + (size_t)P.n * (size_t)P.ldF * esz <= (uintptr_t)base + size;
}

// Layouts worth trying, best predicted first: every split of the resident
// workgroups into solo workers (in steps of 8) and teams of 32 and 16 that gives
// each width it needs a worker, ranked by the largest predicted load.
std::vector<Layout> team_layouts(rac_batch b) {
  bool need32 = false, need16 = false, need1 = false;
  for (int w : b->gwidth) (w == 32 ? need32 : (w == 16 ? need16 : need1)) = true;
  const int R = b->resident;
  std::vector<std::pair<double, Layout>> c;
  for (int ks = need1 ? 8 : 0; ks <= (need1 ? R : 0); ks += 8) {
    const int Rt = R - ks;
    for (int k32 = 0; 32 * k32 <= Rt; ++k32) {
      const int k16 = (Rt - 32 * k32) / 16;
      if ((need32 && k32 == 0) || (need16 && k16 == 0)) continue;
      const int u32 = need32 ? k32 : 0, u16 = need16 ? k16 : 0;
      const double load = std::max(std::max(lpt(b, 32, u32, nullptr), lpt(b, 16, u16, nullptr)),
                                   lpt(b, 1, ks, nullptr));
      c.push_back({load, Layout{u32, u16, ks}});
    }
  }
  std::stable_sort(c.begin(), c.end(), [](const auto& x, const auto& y) { return x.first < y.first; });
  std::vector<Layout> out;
  for (auto& e : c)
    if (std::find(out.begin(), out.end(), e.second) == out.end()) out.push_back(e.second);
  return out;
}

// Use the widths with solo groups (solo = true, the creation layout) or teams only (the
// best predicted team layout).  Groups change arithmetic with their width (a solo group
// sums its products in another order), so the choice must not depend on timing.
rac_status set_widths(rac_batch b, bool solo) {
  if (solo == b->solo_on) return RAC_OK;
  b->gwidth = solo ? b->gw_solo : b->gw_team;
  b->gcost = solo ? b->gc_solo : b->gc_team;
  b->solo_on = solo;
  if (solo) return set_team_layout(b, b->lay0_k32, b->lay0_k16, b->lay0_ks);
  const std::vector<Layout> lay = team_layouts(b);
  if (lay.empty()) return RAC_ERR_UNSUPPORTED;
  return set_team_layout(b, lay[0].k32, lay[0].k16, lay[0].ks);
}

// Whether the solo widths still pay for the lanes that are active.  A solo group holds one
// workgroup for its whole sweep: that pays while many groups share the device, not once
// few remain (a team finishes one group's sweep several times sooner).  Each width set is
// scored by its predicted sweep time, the larger of the active groups' workgroup-time over
// the resident workgroups and the longest active group; teams only are taken when they
// are predicted at least 20% faster.  The decision depends on the lanes' status alone,
// never on the layout or on timing.
rac_status decide_widths(rac_batch b) {
  if (!b->team || !b->solo_on || b->host_active == b->decided_active) return RAC_OK;
  b->decided_active = b->host_active;
  std::vector<int32_t> st(b->nunits, 1);
  BCHK(hipMemcpy2D(st.data(), sizeof(int32_t), &b->A.sc[0].status, sizeof(DevScalars), sizeof(int32_t),
                   b->nunits, hipMemcpyDeviceToHost));
  double area_s = 0.0, long_s = 0.0, area_t = 0.0, long_t = 0.0;
  for (size_t g = 0; g < b->hgroups.size(); ++g) {
    const TGroup& G = b->hgroups[g];
    bool any = false;
    for (int q = 0; q < G.nl; ++q) any |= st[G.lane[q]] == 0;
    if (!any) continue;
    area_s += b->gw_solo[g] * b->gc_solo[g];
    long_s = std::max(long_s, b->gc_solo[g]);
    area_t += b->gw_team[g] * b->gc_team[g];
    long_t = std::max(long_t, b->gc_team[g]);
  }
  const double R = (double)b->resident;
  const double t_solo = std::max(area_s / R, long_s), t_team = std::max(area_t / R, long_t);
  return t_team < 0.8 * t_solo ? set_widths(b, false) : RAC_OK;
}

// Time one chunk with each of the best predicted team layouts (from the same
// state) and keep the fastest.
rac_status autotune_team(rac_batch b) {
  const std::string path = tune_cache_path();
  std::vector<Layout> cand = team_layouts(b);
  if (cand.size() > 3) cand.resize(3);
  if (FILE* f = std::fopen(path.c_str(), "r")) {
    char line[640], key[512];
    int a = 0, c = 0, d = 0;
    while (std::fgets(line, sizeof(line), f))
      if (std::sscanf(line, "%511s %d %d %d", key, &a, &c, &d) == 4)
        for (auto& cd : cand)
          if (b->tune_key == key && cd.k32 == a && cd.k16 == c && cd.ks == d) {
            std::fclose(f);
            return set_team_layout(b, a, c, d);
          }
    std::fclose(f);
  }
  Snapshot snap;
  rac_status r = state_copy(b, true, snap);
  if (r != RAC_OK) return r;
  hipEvent_t e0, e1;
  BCHK(hipEventCreate(&e0));
  BCHK(hipEventCreate(&e1));
  float best = 1e30f;
  Layout pick = cand[0];
  for (auto& cd : cand) {
    r = set_team_layout(b, cd.k32, cd.k16, cd.ks);
    if (r != RAC_OK) return r;
    BCHK(hipEventRecord(e0, b->cs));
    r = enqueue_chunk(b, b->T, b->cs);
    if (r != RAC_OK) return r;
    BCHK(hipEventRecord(e1, b->cs));
    BCHK(hipEventSynchronize(e1));
    uint32_t aborted = 0;
    BCHK(hipMemcpy(&aborted, b->TA.abort_flag, sizeof(uint32_t), hipMemcpyDeviceToHost));
    if (aborted) return RAC_ERR_DEVICE;
    float ms = 0.f;
    BCHK(hipEventElapsedTime(&ms, e0, e1));
    if (ms < best) { best = ms; pick = cd; }
    r = state_copy(b, false, snap);
    if (r != RAC_OK) return r;
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (FILE* f = std::fopen(path.c_str(), "a")) {
    std::fprintf(f, "%s %d %d %d\n", b->tune_key.c_str(), pick.k32, pick.k16, pick.ks);
    std::fclose(f);
  }
  return set_team_layout(b, pick.k32, pick.k16, pick.ks);
}

// Time one chunk with each sweep row unroll on this batch (from the same
// state), keep the fastest, and remember it per batch shape.
rac_status autotune(rac_batch b) {
  const std::string path = tune_cache_path();
  if (FILE* f = std::fopen(path.c_str(), "r")) {
    char line[640], key[512];
    int un = 0;
    while (std::fgets(line, sizeof(line), f))
      if (std::sscanf(line, "%511s %d", key, &un) == 2 && b->tune_key == key && (un == 1 || un == 2 || un == 4)) {
        b->A.unroll = un;
        std::fclose(f);
        return RAC_OK;
      }
    std::fclose(f);
  }
  Snapshot snap;
  rac_status r = state_copy(b, true, snap);
  if (r != RAC_OK) return r;
  hipEvent_t e0, e1;
  BCHK(hipEventCreate(&e0));
  BCHK(hipEventCreate(&e1));
  float best = 1e30f;
  int best_un = 2;
  for (int un : {1, 2, 4}) {
    b->A.unroll = un;
    BCHK(hipEventRecord(e0, b->cs));
    r = enqueue_chunk(b, b->T, b->cs);
    if (r != RAC_OK) return r;
    BCHK(hipEventRecord(e1, b->cs));
    BCHK(hipEventSynchronize(e1));
    float ms = 0.f;
    BCHK(hipEventElapsedTime(&ms, e0, e1));
    if (ms < best) { best = ms; best_un = un; }
    r = state_copy(b, false, snap);
    if (r != RAC_OK) return r;
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  b->A.unroll = best_un;
  if (FILE* f = std::fopen(path.c_str(), "a")) {
    std::fprintf(f, "%s %d\n", b->tune_key.c_str(), best_un);
    std::fclose(f);
  }
  return RAC_OK;
}

}  // namespace

extern "C" {

rac_status rac_batch_create(int32_t ninst, const rac_problem* inst, int32_t nlanes, const rac_lane* lanes,
                            const rac_batch_opts* opts, rac_batch* out) {
  if (!out || !opts || !inst || !lanes || ninst < 1 || nlanes < 1) return RAC_ERR_ARG;
  *out = nullptr;
  rac_batch_opts O = *opts;
  if (O.block_size < 1 || O.block_size > 64) return RAC_ERR_ARG;
  if (O.check_every < 1 || O.max_iter < 0 || !std::isfinite(O.tol) || O.tol < 0.0) return RAC_ERR_ARG;
  if (O.precision != RAC_PREC_FP64 && O.precision != RAC_PREC_MIXED) return RAC_ERR_ARG;
  if (O.beta_mode != RAC_BETA_FIXED && O.beta_mode != RAC_BETA_RESBAL && O.beta_mode != RAC_BETA_MLP)
    return RAC_ERR_ARG;
  if (O.beta_mode == RAC_BETA_MLP && !O.mlp_weights) return RAC_ERR_ARG;
  if (O.sweep != RAC_BSWEEP_AUTO && O.sweep != RAC_BSWEEP_LANE && O.sweep != RAC_BSWEEP_TEAM) return RAC_ERR_ARG;
  if (O.rb_mu <= 0.0) O.rb_mu = 10.0;
  if (O.rb_tau <= 0.0) O.rb_tau = 2.0;
  if (!(O.mlp_ymax > 0.0)) O.mlp_ymax = std::log(10.0);
  const int32_t dtype = inst[0].F_dtype;
  int64_t maxn = 0;
  for (int i = 0; i < ninst; ++i) {
    const rac_problem& P = inst[i];
    if (P.Hd || P.meq != 0 || P.A || P.colptr) return RAC_ERR_UNSUPPORTED;   // dense and sparse forms: single instance
    if (P.n < 1 || P.rows < 1 || !P.F || P.ldF < P.rows || !P.c || P.F_dtype != dtype) return RAC_ERR_ARG;
    if (P.n > 8192 || !std::isfinite(P.Ns) || !(P.Ns > 0.0) || !std::isfinite(P.b)) return RAC_ERR_ARG;
    if (dtype != RAC_DT_F64 && dtype != RAC_DT_F32 && dtype != RAC_DT_BF16) return RAC_ERR_ARG;
    if (P.n > maxn) maxn = P.n;
  }
  for (int i = 0; i < ninst; ++i) {
    const rac_status v = check_problem_arrays(inst[i]);   // no NaN or infinity in the device arrays
    if (v != RAC_OK) return v;
  }
  for (int u = 0; u < nlanes; ++u) {
    const rac_lane& L = lanes[u];
    if (L.problem < 0 || L.problem >= ninst || !std::isfinite(L.beta0) || !(L.beta0 > 0.0)) return RAC_ERR_ARG;
    if (L.prox < RAC_PROX_NONE || L.prox > RAC_PROX_BOX) return RAC_ERR_ARG;
    if (L.prox == RAC_PROX_ELASTIC_NET &&
        (!std::isfinite(L.lambda) || L.lambda < 0.0 || !(L.alpha >= 0.0 && L.alpha <= 1.0)))
      return RAC_ERR_ARG;
    const rac_problem& P = inst[L.problem];
    if (L.prox == RAC_PROX_BOX && !(P.lo <= P.hi)) return RAC_ERR_ARG;
  }
  // the caller's pending work (e.g. the kernels that produced F) completes before
  // any of the batch's own streams touches the data
  if (hipDeviceSynchronize() != hipSuccess) return RAC_ERR_DEVICE;
  rac_batch b = new (std::nothrow) rac_batch_s();
  if (!b) return RAC_ERR_NOMEM;
  auto fail = [&](rac_status r) {
    b->buf.release();
    if (b->gexec) (void)hipGraphExecDestroy(b->gexec);
    if (b->graph) (void)hipGraphDestroy(b->graph);
    if (b->ev) (void)hipEventDestroy(b->ev);
    if (b->cs) (void)hipStreamDestroy(b->cs);
    delete b;
    return r;
  };
  b->O = O;
  b->ninst = ninst;
  b->nunits = nlanes;
  b->T = (int)O.check_every;
  const int64_t s = O.block_size;
  b->SP = s <= 16 ? 16 : (s <= 32 ? 32 : 64);
  // instances: partitions (T per instance) and block Grams
  int64_t poff = 0, goff = 0, rows_sum = 0;
  std::vector<int2> gt;
  for (int i = 0; i < ninst; ++i) {
    const rac_problem& P = inst[i];
    BInst I{};
    I.F = P.F; I.ldF = P.ldF; I.rows = P.rows; I.n = P.n; I.p = (P.n + s - 1) / s;
    I.poff = poff; I.goff = goff; I.key_instance = (uint64_t)i;
    const int vw = 16 / (dtype == RAC_DT_F64 ? 8 : (dtype == RAC_DT_F32 ? 4 : 2));
    I.vec = (P.ldF % vw == 0) && ((uintptr_t)P.F % 16 == 0);
    for (int64_t q = 0; q < I.p; ++q) gt.push_back(make_int2(i, (int)q));
    poff += (int64_t)b->T * P.n;
    goff += I.p;
    b->hinst.push_back(I);
  }
  // lanes
  int64_t xoff = 0, uoff = 0, moff = 0;
  std::vector<int2> it;
  int64_t maxp = 0;
  for (int u = 0; u < nlanes; ++u) {
    const rac_lane& L = lanes[u];
    const rac_problem& P = inst[L.problem];
    const BInst& I = b->hinst[L.problem];
    BUnit U{};
    U.F = P.F; U.ldF = P.ldF; U.rows = P.rows; U.n = P.n; U.p = I.p; U.Ns = P.Ns;
    U.h = P.h; U.c = P.c; U.a = P.a; U.b = P.b; U.prox = L.prox; U.inst = L.problem;
    U.lam = L.lambda; U.alpha = L.alpha; U.lo = P.lo; U.hi = P.hi;
    U.xoff = xoff; U.uoff = uoff; U.goff = I.goff; U.moff = moff; U.poff = I.poff;
    for (int64_t q = 0; q < I.p; ++q) it.push_back(make_int2(u, (int)q));
    xoff += P.n;
    uoff += P.rows;
    moff += I.p;
    rows_sum += P.rows;
    if (I.p > maxp) maxp = I.p;
    b->hunit.push_back(U);
  }
  // Gram tasks of the longest columns first: one workgroup streams a whole block, so the
  // largest instances set the phase's tail unless they start early (the order leaves
  // every result unchanged)
  std::stable_sort(gt.begin(), gt.end(), [&](const int2& x, const int2& y) {
    return inst[x.x].rows > inst[y.x].rows;
  });
  b->ngt = (int)gt.size();
  BatchArgs& A = b->A;
  A.dtype = dtype; A.sp = b->SP; A.T = b->T; A.nunits = nlanes; A.ninst = ninst;
  int np2 = 1;
  while (np2 < maxn) np2 <<= 1;
  A.np2 = np2;
  A.seed = O.seed;
  A.ninv = (int)it.size();
  A.KC = (int)((maxn + 63) / 64);
  A.beta_mode = O.beta_mode; A.rb_mu = O.rb_mu; A.rb_tau = O.rb_tau; A.tol = O.tol;
  A.mlp_w = O.mlp_weights; A.mlp_ymax = O.mlp_ymax;
  A.unroll = 2;
  const size_t ss = (size_t)b->SP * b->SP;
  // A Gram and inverse slot per iteration of a chunk while they take at most an eighth
  // of the device memory and half of what is free (RACMB_ASSEMBLY_SLOTS=1: one slot)
  int nslot = 1;
  {
    size_t mfree = 0, mtotal = 0;
    const double per = (double)(goff + moff) * (double)ss * sizeof(double);
    const char* es = std::getenv("RACMB_ASSEMBLY_SLOTS");
    const bool one = es && std::atoi(es) == 1;
    if (!one && b->T > 1 && hipMemGetInfo(&mfree, &mtotal) == hipSuccess &&
        per * b->T <= (double)mtotal / 8 && per * b->T <= (double)mfree / 2)
      nslot = b->T;
    (void)hipGetLastError();
  }
  b->nslot = nslot;
  A.gslot = nslot > 1 ? (int64_t)(goff * ss) : 0;
  A.mslot = nslot > 1 ? (int64_t)(moff * ss) : 0;
  bool ok = b->buf.alloc(&b->dinst, ninst) && b->buf.alloc(&b->dunit, nlanes) &&
            b->buf.alloc(&b->gtasks, gt.size()) && b->buf.alloc(const_cast<int2**>(&A.inv_tasks), it.size()) &&
            b->buf.alloc(&A.perm, poff) && b->buf.alloc(const_cast<double**>(&A.G), goff * ss * nslot) &&
            b->buf.alloc(&A.Minv, moff * ss * nslot) && b->buf.alloc(&A.X, xoff) && b->buf.alloc(&A.Z, xoff) &&
            b->buf.alloc(&A.XI, xoff) && b->buf.alloc(&A.ZP, xoff) && b->buf.alloc(&A.U, uoff) &&
            b->buf.alloc(&A.sc, nlanes) && b->buf.alloc(&A.kpart, (size_t)nlanes * A.KC * 10) &&
            b->buf.alloc(&A.inst_active, ninst) && b->buf.alloc(&A.nactive, 1) && b->buf.alloc(&A.kdev, 1);
  if (!ok) return fail(RAC_ERR_NOMEM);
  A.inst = b->dinst;
  A.units = b->dunit;
  std::vector<DevScalars> hs;
  for (int u = 0; u < nlanes; ++u) hs.push_back(fresh(lanes[u].beta0));
  std::vector<int32_t> act(ninst, 1);
  const int32_t nact = nlanes;
  const int64_t k0 = 0;
  if (hipMemcpy(b->dinst, b->hinst.data(), sizeof(BInst) * ninst, hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(b->dunit, b->hunit.data(), sizeof(BUnit) * nlanes, hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(b->gtasks, gt.data(), sizeof(int2) * gt.size(), hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(const_cast<int2*>(A.inv_tasks), it.data(), sizeof(int2) * it.size(), hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(A.sc, hs.data(), sizeof(DevScalars) * nlanes, hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(A.inst_active, act.data(), sizeof(int32_t) * ninst, hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(A.nactive, &nact, sizeof(int32_t), hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(A.kdev, &k0, sizeof(int64_t), hipMemcpyHostToDevice) != hipSuccess ||
      hipMemset(A.X, 0, sizeof(double) * xoff) != hipSuccess || hipMemset(A.Z, 0, sizeof(double) * xoff) != hipSuccess ||
      hipMemset(A.XI, 0, sizeof(double) * xoff) != hipSuccess || hipMemset(A.ZP, 0, sizeof(double) * xoff) != hipSuccess ||
      hipMemset(A.U, 0, sizeof(double) * uoff) != hipSuccess)
    return fail(RAC_ERR_DEVICE);
  b->host_active = nlanes;
  // ---- team sweep: lane groups (up to 16 lanes of one instance), each run by a
  // team of 16 workgroups when the instance's rows fit 16 members, else of 32
  if (O.sweep != RAC_BSWEEP_LANE) {
    std::vector<std::vector<int>> by_inst(ninst);
    for (int u = 0; u < nlanes; ++u) by_inst[lanes[u].problem].push_back(u);
    const int ntmax = dtype == RAC_DT_BF16 ? 10 : 8;
    auto member_rows = [](int64_t rows, int w) { return (rows + w - 1) / w + 15; };   // bound on a member's rows
    bool fits = true;
    int64_t need = 0;
    std::vector<int> width(ninst, 0);
    int64_t solo_rows = kSoloRows;
    if (const char* e = std::getenv("RACMB_SOLO_ROWS")) solo_rows = std::atoll(e);
    // Predicted time of one of a group's blocks (us): a team's exchanges plus its member's
    // products, or a solo workgroup's products over all rows and its solves (both measured).
    auto block_cost = [](int64_t rows, int w) {
      return w == 1 ? 28.0 + 29.0 * (double)rows / 1000.0 : 14.0 + 12.0 * (double)((rows + w - 1) / w) / 640.0;
    };
    // Candidates for solo groups: at most solo_rows rows, laid out for the clamped vector
    // loads.  A solo group holds one workgroup for the whole sweep, so none may take longer
    // than the predicted sweep: while the longest solo group exceeds the larger of the
    // workgroup-time bound (all groups' workgroup-time over the resident workgroups) and
    // the longest team group, its instance goes to a team instead.
    std::vector<int> wteam(ninst, 0);
    std::vector<char> solo(ninst, 0);
    for (int i = 0; i < ninst; ++i) {
      if (by_inst[i].empty()) continue;
      wteam[i] = member_rows(inst[i].rows, 16) <= 64 * ntmax ? 16 : 32;
      solo[i] = inst[i].rows <= solo_rows && solo_layout_ok(inst[i]);
    }
    const double rw_all = (double)std::max(1, tsweep_max_resident(dtype, ntmax));
    const char* force = std::getenv("RACMB_SOLO_FORCE");   // every candidate solo (tests of the solo path)
    for (;;) {
      if (force && *force == '1') break;
      double area = 0.0, longest_team = 0.0, worst = 0.0;
      int wi = -1;
      for (int i = 0; i < ninst; ++i) {
        if (by_inst[i].empty()) continue;
        const double ng = (double)((by_inst[i].size() + 15) / 16), p_i = (double)b->hinst[i].p;
        const int w = solo[i] ? 1 : wteam[i];
        const double c = p_i * block_cost(inst[i].rows, w);
        area += ng * w * c;
        if (!solo[i]) longest_team = std::max(longest_team, c);
      }
      const double bound = std::max(area / rw_all, longest_team);
      for (int i = 0; i < ninst; ++i) {
        if (!solo[i]) continue;
        const double c = (double)b->hinst[i].p * block_cost(inst[i].rows, 1);
        if (c > bound && c > worst) { worst = c; wi = i; }
      }
      if (wi < 0) break;
      solo[wi] = 0;
    }
    for (int i = 0; i < ninst; ++i) {       // the tiles a member needs: every instance may run on a team
      if (by_inst[i].empty()) continue;
      width[i] = solo[i] ? 1 : wteam[i];     // solo: one workgroup streams the whole instance
      if (member_rows(inst[i].rows, wteam[i]) > 64 * ntmax) fits = false;
      need = std::max<int64_t>(need, member_rows(inst[i].rows, wteam[i]));
    }
    const int NT = need <= 64 * 8 ? 8 : ntmax;
    const int resident = fits ? tsweep_max_resident(dtype, NT) : 0;
    if (resident >= 32) {
      const int esz = dtype == RAC_DT_F64 ? 8 : (dtype == RAC_DT_F32 ? 4 : 2);
      for (int i = 0; i < ninst; ++i) {
        if (by_inst[i].empty()) continue;
        const rac_problem& P = inst[i];
        const int vec4 = (P.ldF % 4 == 0) && ((uintptr_t)P.F % (uintptr_t)(4 * esz) == 0);
        const int vec8 = (P.ldF % 8 == 0) && ((uintptr_t)P.F % 16 == 0);
        const int span = solo_layout_ok(P) ? 1 : 0;
        const double cost = (double)b->hinst[i].p * block_cost(P.rows, width[i]);
        const double cost_team = (double)b->hinst[i].p * block_cost(P.rows, wteam[i]);
        for (size_t g0 = 0; g0 < by_inst[i].size(); g0 += 16) {
          TGroup G{};
          G.inst = i;
          G.nl = (int32_t)std::min<size_t>(16, by_inst[i].size() - g0);
          G.vec4 = vec4;
          G.vec8 = vec8;
          G.span = span;
          for (int q = 0; q < 16; ++q) G.lane[q] = q < G.nl ? by_inst[i][g0 + q] : -1;
          b->hgroups.push_back(G);
          b->gcost.push_back(cost);
          b->gwidth.push_back(width[i]);
          b->gw_solo.push_back(width[i]);
          b->gw_team.push_back(wteam[i]);
          b->gc_solo.push_back(cost);
          b->gc_team.push_back(cost_team);
          if (width[i] == 1) b->solo_on = true;
        }
      }
      const int ng = (int)b->hgroups.size();
      const int maxt = resident;   // at most one team (or solo worker) per workgroup
      b->resident = resident;
      b->max_teams = maxt;
      b->TA.NT = NT;
      ok = b->buf.alloc(&b->dgroups, ng) && b->buf.alloc(&b->dteam_off, maxt + 1) &&
           b->buf.alloc(&b->dteam_list, ng) && b->buf.alloc(&b->dteam_w, maxt) &&
           b->buf.alloc(&b->dteam_part, maxt) && b->buf.alloc(&b->dblk_team, resident) &&
           b->buf.alloc(&b->dblk_member, resident) && b->buf.alloc(&b->TA.part, (size_t)resident * 2 * 1024) &&
           b->buf.alloc(&b->TA.delta, (size_t)maxt * 2 * 1024) && b->buf.alloc(&b->TA.flags, (size_t)maxt * 128) &&
           b->buf.alloc(&b->TA.abort_flag, 1);
      if (!ok) return fail(RAC_ERR_NOMEM);
      // Grouped KKT tasks (group, pair of 64-column chunks).  Workgroups go to the eight XCDs in
      // turn (workgroup k to XCD k mod 8), so the chunks of a group are dealt to one
      // XCD's queue (its u is then read into one L2), the largest groups first onto the
      // least loaded queue, and the queues are interleaved (an exhausted queue's turns
      // are empty tasks, group -1, that keep the others on their XCDs); the order leaves
      // every result unchanged.
      std::vector<int2> kt;
      {
        std::vector<int> order(ng);
        for (int g = 0; g < ng; ++g) order[g] = g;
        auto rows_of = [&](int g) { return inst[b->hgroups[g].inst].rows; };
        std::stable_sort(order.begin(), order.end(), [&](int x, int y) { return rows_of(x) > rows_of(y); });
        std::vector<std::vector<int2>> xq(8);
        std::vector<double> load(8, 0.0);
        for (int g : order) {
          const int64_t nch = (inst[b->hgroups[g].inst].n + 127) / 128;
          const int x = (int)(std::min_element(load.begin(), load.end()) - load.begin());
          for (int64_t ch = 0; ch < nch; ++ch) xq[x].push_back(make_int2(g, (int)ch));
          load[x] += (double)nch * (double)rows_of(g);
        }
        size_t len = 0;
        for (int x = 0; x < 8; ++x) len = std::max(len, xq[x].size());
        for (size_t k = 0; k < len; ++k)
          for (int x = 0; x < 8; ++x) kt.push_back(k < xq[x].size() ? xq[x][k] : make_int2(-1, 0));
      }
      b->nkkt_tasks = (int)kt.size();
      if (!b->buf.alloc(&b->dkkt_tasks, kt.size())) return fail(RAC_ERR_NOMEM);
      if (hipMemcpy(b->dkkt_tasks, kt.data(), sizeof(int2) * kt.size(), hipMemcpyHostToDevice) != hipSuccess ||
          hipMemcpy(b->dgroups, b->hgroups.data(), sizeof(TGroup) * ng, hipMemcpyHostToDevice) != hipSuccess ||
          hipMemset(b->TA.abort_flag, 0, sizeof(uint32_t)) != hipSuccess ||
          hipMemset(b->TA.delta, 0, sizeof(double) * (size_t)maxt * 2 * 1024) != hipSuccess)
        return fail(RAC_ERR_DEVICE);
      b->TA.groups = b->dgroups;
      b->TA.team_off = b->dteam_off;
      b->TA.team_list = b->dteam_list;
      b->TA.team_w = b->dteam_w;
      b->TA.team_part = b->dteam_part;
      b->TA.blk_team = b->dblk_team;
      b->TA.blk_member = b->dblk_member;
      b->team = true;
      const std::vector<Layout> lay = team_layouts(b);
      if (lay.empty()) return fail(RAC_ERR_UNSUPPORTED);
      const rac_status r = set_team_layout(b, lay[0].k32, lay[0].k16, lay[0].ks);
      if (r != RAC_OK) return fail(r);
    } else if (O.sweep == RAC_BSWEEP_TEAM) {
      return fail(RAC_ERR_UNSUPPORTED);
    }
  }
  if (hipStreamCreateWithFlags(&b->cs, hipStreamNonBlocking) != hipSuccess) return fail(RAC_ERR_DEVICE);
  if (hipEventCreateWithFlags(&b->ev, hipEventDisableTiming) != hipSuccess) return fail(RAC_ERR_DEVICE);
  char key[256];
  if (b->team) {
    int n32 = 0, n1 = 0;
    for (int w : b->gwidth) { n32 += w == 32; n1 += w == 1; }
    std::snprintf(key, sizeof(key), "tsweep3:dt%d:sp%d:lanes%d:groups%d:g32_%d:g1_%d:rows%lld:NT%d:R%d:T%d:gfx950",
                  dtype, b->SP, nlanes, (int)b->hgroups.size(), n32, n1, (long long)(rows_sum / 1024), b->TA.NT,
                  b->resident, b->T);
  }
  else
    std::snprintf(key, sizeof(key), "bsweep:dt%d:sp%d:lanes%d:rows%lld:T%d:gfx950", dtype, b->SP, nlanes,
                  (long long)(rows_sum / 1024), b->T);
  b->tune_key = key;
  if (O.tune) {
    rac_status r = b->team ? autotune_team(b) : autotune(b);
    if (r != RAC_OK) return fail(r);
  }
  b->lay0_k32 = b->k32;
  b->lay0_k16 = b->k16;
  b->lay0_ks = b->ks;
  b->decided_active = b->host_active;
  if (hipDeviceSynchronize() != hipSuccess) return fail(RAC_ERR_DEVICE);
  *out = b;
  return RAC_OK;
}

rac_status rac_batch_destroy(rac_batch b) {
  if (!b) return RAC_ERR_ARG;
  (void)hipDeviceSynchronize();
  if (b->gexec) (void)hipGraphExecDestroy(b->gexec);
  if (b->graph) (void)hipGraphDestroy(b->graph);
  if (b->ev) (void)hipEventDestroy(b->ev);
  for (hipEvent_t e : b->ev_t) (void)hipEventDestroy(e);
  if (b->cs) (void)hipStreamDestroy(b->cs);
  b->buf.release();
  delete b;
  return RAC_OK;
}

rac_status rac_batch_set_timing(rac_batch b, int32_t enable) {
  if (!b) return RAC_ERR_ARG;
  BCHK(hipStreamSynchronize(b->cs));
  b->timing = enable != 0;
  b->ev_phase.clear();
  for (int q = 0; q < RAC_NUM_PHASES; ++q) { b->phase_ms[q] = 0.0; b->phase_count[q] = 0; }
  return RAC_OK;
}

rac_status rac_batch_timing(rac_batch b, double* ms, int64_t* launches) {
  if (!b || !ms) return RAC_ERR_ARG;
  for (int q = 0; q < RAC_NUM_PHASES; ++q) {
    ms[q] = b->phase_ms[q];
    if (launches) launches[q] = b->phase_count[q];
  }
  return RAC_OK;
}

rac_status rac_batch_run(rac_batch b, void* stream, int64_t* iters, int32_t* active) {
  if (!b) return RAC_ERR_ARG;
  hipStream_t st = (hipStream_t)stream;
  // the batch's stream starts after the caller's prior work and the caller waits for it at the end
  BCHK(hipEventRecord(b->ev, st));
  BCHK(hipStreamWaitEvent(b->cs, b->ev, 0));
  int64_t done = 0;
  while (done < b->O.max_iter && b->host_active > 0) {
    const int Tc = (int)std::min<int64_t>(b->T, b->O.max_iter - done);
    if (b->O.use_graph && Tc == b->T && !b->timing) {
      if (!b->gexec) {
        BCHK(hipStreamBeginCapture(b->cs, hipStreamCaptureModeThreadLocal));
        rac_status r = enqueue_chunk(b, Tc, b->cs);
        hipGraph_t g = nullptr;
        hipError_t e = hipStreamEndCapture(b->cs, &g);
        if (r != RAC_OK) return r;
        BCHK(e);
        b->graph = g;
        BCHK(hipGraphInstantiate(&b->gexec, g, nullptr, nullptr, 0));
      }
      BCHK(hipGraphLaunch(b->gexec, b->cs));
      b->graph_used = true;
    } else {
      rac_status r = enqueue_chunk(b, Tc, b->cs);
      if (r != RAC_OK) return r;
    }
    BCHK(hipMemcpyAsync(&b->host_active, b->A.nactive, sizeof(int32_t), hipMemcpyDeviceToHost, b->cs));
    uint32_t aborted = 0;
    if (b->team) BCHK(hipMemcpyAsync(&aborted, b->TA.abort_flag, sizeof(uint32_t), hipMemcpyDeviceToHost, b->cs));
    BCHK(hipStreamSynchronize(b->cs));
    if (aborted) return RAC_ERR_DEVICE;   // a team exchange timed out
    {
      const rac_status r = collect_timing(b);
      if (r != RAC_OK) return r;
    }
    done += Tc;
    {
      const rac_status r = decide_widths(b);
      if (r != RAC_OK) return r;
    }
  }
  b->k += done;
  BCHK(hipEventRecord(b->ev, b->cs));
  BCHK(hipStreamWaitEvent(st, b->ev, 0));
  if (iters) *iters = done;
  if (active) *active = b->host_active;
  return RAC_OK;
}

rac_status rac_batch_lane(rac_batch b, int32_t lane, rac_result* res, double* x, double* z, double* xi) {
  if (!b || lane < 0 || lane >= b->nunits) return RAC_ERR_ARG;
  const BUnit& U = b->hunit[lane];
  BCHK(hipStreamSynchronize(b->cs));
  DevScalars h;
  BCHK(hipMemcpy(&h, b->A.sc + lane, sizeof(DevScalars), hipMemcpyDeviceToHost));
  const size_t nb = sizeof(double) * U.n;
  if (x) BCHK(hipMemcpy(x, b->A.X + U.xoff, nb, hipMemcpyDeviceToDevice));
  if (z) BCHK(hipMemcpy(z, b->A.Z + U.xoff, nb, hipMemcpyDeviceToDevice));
  if (xi) BCHK(hipMemcpy(xi, b->A.XI + U.xoff, nb, hipMemcpyDeviceToDevice));
  if (res) {
    std::memset(res, 0, sizeof(*res));
    res->iters = h.k;
    res->status = h.status == 1 ? RAC_RUN_CONVERGED : (h.status == 2 ? RAC_RUN_DIVERGED : RAC_RUN_MAX_ITER);
    res->kkt = h.kkt;
    res->beta = h.beta;
    res->objective = NAN;
    res->fail_iter = h.fail_key == ~0ULL ? -1 : (int64_t)(h.fail_key >> 32);
    res->fail_block = h.fail_key == ~0ULL ? -1 : (int64_t)(h.fail_key & 0xffffffffULL);
  }
  return h.fail_key == ~0ULL ? RAC_OK : RAC_ERR_NOT_PD;
}

rac_status rac_batch_state_export(rac_batch b, void* buf, size_t* bytes) {
  if (!b || !bytes) return RAC_ERR_ARG;
  const size_t need = sizeof(BatchStateHeader) + state_bytes(b);
  if (!buf) {
    *bytes = need;
    return RAC_OK;
  }
  if (*bytes < need) return RAC_ERR_ARG;
  BCHK(hipStreamSynchronize(b->cs));
  BatchStateHeader h{kBatchStateMagic, b->nunits, b->ninst, (int64_t)state_bytes(b), b->k,
                     (int64_t)sizeof(DevScalars), b->solo_on ? 1 : 0};
  std::memcpy(buf, &h, sizeof(h));
  const rac_status r = state_xfer(b, true, (char*)buf + sizeof(h));
  if (r != RAC_OK) return r;
  *bytes = need;
  return RAC_OK;
}

rac_status rac_batch_state_import(rac_batch b, const void* buf, size_t bytes) {
  if (!b || !buf || bytes < sizeof(BatchStateHeader)) return RAC_ERR_ARG;
  BatchStateHeader h;
  std::memcpy(&h, buf, sizeof(h));
  if (h.magic != kBatchStateMagic || h.nunits != b->nunits || h.ninst != b->ninst ||
      h.state_bytes != (int64_t)state_bytes(b) || h.scalars_bytes != (int64_t)sizeof(DevScalars) ||
      bytes < sizeof(h) + (size_t)h.state_bytes)
    return RAC_ERR_ARG;
  BCHK(hipStreamSynchronize(b->cs));
  const rac_status r = state_xfer(b, false, const_cast<char*>((const char*)buf) + sizeof(h));
  if (r != RAC_OK) return r;
  b->k = h.k;
  BCHK(hipMemcpy(&b->host_active, b->A.nactive, sizeof(int32_t), hipMemcpyDeviceToHost));
  b->decided_active = b->host_active;
  if (b->team && h.solo_on != (b->solo_on ? 1 : 0)) {   // the widths the exporting batch used
    if (h.solo_on && b->gw_solo == b->gw_team) return RAC_ERR_ARG;
    return set_widths(b, h.solo_on != 0);
  }
  return RAC_OK;
}

rac_status rac_batch_set_lane_state(rac_batch b, int32_t lane, const double* x, const double* z, const double* xi,
                                    double mu, double beta) {
  if (!b || lane < 0 || lane >= b->nunits || !x || !z || !xi || !std::isfinite(mu) || !std::isfinite(beta) ||
      !(beta > 0.0))
    return RAC_ERR_ARG;
  const BUnit& U = b->hunit[lane];
  BCHK(hipStreamSynchronize(b->cs));
  DevScalars h;
  BCHK(hipMemcpy(&h, b->A.sc + lane, sizeof(DevScalars), hipMemcpyDeviceToHost));
  if (h.status != 0) return RAC_ERR_ARG;   // a retired lane stays retired
  const size_t nb = sizeof(double) * U.n;
  BCHK(hipMemcpy(b->A.X + U.xoff, x, nb, hipMemcpyDeviceToDevice));
  BCHK(hipMemcpy(b->A.Z + U.xoff, z, nb, hipMemcpyDeviceToDevice));
  BCHK(hipMemcpy(b->A.XI + U.xoff, xi, nb, hipMemcpyDeviceToDevice));
  BCHK(hipMemcpy(b->A.ZP + U.xoff, z, nb, hipMemcpyDeviceToDevice));
  // the lane's residuals u = F x and t = a'x for its instance's data
  const int np = (int)std::min<int64_t>(64, std::max<int64_t>(1, (U.n + 255) / 256));
  double *part = nullptr, *red = nullptr, *tv = nullptr;
  uint32_t* done = nullptr;
  DevBufs tmp;
  if (!tmp.alloc(&part, (size_t)np * U.rows) || !tmp.alloc(&red, (size_t)kRedSlots) || !tmp.alloc(&tv, 1) ||
      !tmp.alloc(&done, 4)) {
    tmp.release();
    return RAC_ERR_NOMEM;
  }
  hipError_t e = hipMemset(done, 0, 4 * sizeof(uint32_t));
  if (e == hipSuccess) e = hipMemset(tv, 0, sizeof(double));
  if (e == hipSuccess)
    e = launch_matvec_F_parts(U.F, b->A.dtype, U.ldF, U.rows, U.n, b->A.X + U.xoff, b->A.U + U.uoff, part, np,
                              b->cs);
  if (e == hipSuccess && U.a) e = launch_dot_red(U.a, b->A.X + U.xoff, U.n, red, done, tv, b->cs);
  if (e == hipSuccess) e = hipStreamSynchronize(b->cs);
  double t = 0.0;
  if (e == hipSuccess) e = hipMemcpy(&t, tv, sizeof(double), hipMemcpyDeviceToHost);
  tmp.release();
  if (e != hipSuccess) return RAC_ERR_DEVICE;
  DevScalars f = fresh(beta);
  f.mu = mu;
  f.t = t;
  BCHK(hipMemcpy(b->A.sc + lane, &f, sizeof(DevScalars), hipMemcpyHostToDevice));
  return RAC_OK;
}

rac_status rac_batch_info(rac_batch b, int64_t* info) {
  if (!b || !info) return RAC_ERR_ARG;
  info[0] = b->nunits;
  info[1] = b->ninst;
  info[2] = b->ngt;
  info[3] = b->A.ninv;
  info[4] = b->A.unroll;
  info[5] = b->graph_used ? 1 : 0;
  info[6] = b->team ? (b->k32 > 0 ? 32 : (b->k16 > 0 ? 16 : 1)) : 0;
  info[7] = b->team ? b->TA.nteams : 0;
  info[8] = b->team ? (int64_t)std::count(b->gwidth.begin(), b->gwidth.end(), 1) : 0;
  info[9] = b->nslot;
  return RAC_OK;
}

}  // extern "C"
