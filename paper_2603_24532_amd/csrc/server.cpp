// Continuous-batching server for EOS-point requests (see include/mbpt_vegas.h).
//
// Layout of the caller's workspace: a slot table (TaskDev, grid, histogram and
// iteration-log ring per slot), a descriptor table (kDiagsPerSlot DiagDev
// entries per slot on average; a diagram group's members take consecutive
// entries), parallel per-work-item regions (partial sums, counters and, with
// regularised components, component sums) indexed by a storage index, and a
// byte arena for the isospin groups and label terms of each resident request.
// Descriptor entries, storage-index ranges and arena bytes are handed out
// first-fit and returned at retirement; all three are bookkept on the host.
//
// One round (mbpt_server_step): admit queued requests in arrival order while a
// slot is free and there is room for the head request's items and terms; run
// the planned VEGAS iterations of every resident request, each iteration one
// sample launch per order present (over the work items of all of that order's
// requests) plus the iteration-end launch; copy the task states back; retire
// requests whose sigma reached max(sigma_rel |E|, sigma_abs) after at least
// kMinIters iterations, or whose evaluations reached max_evals.  With
// regularised components (fixed at creation from the context) the host
// combines each request's per-iteration component estimates, read back from
// the slot's log ring every step, and the target applies to the
// extrapolation to zero shift.  A request
// samples its own Philox stream (key = ticket), so its result does not depend
// on what else is resident.  Requests run through the spin x isospin kernel; a
// neutron-matter request runs at proton fraction 0, where that label sum equals
// the spin-only one sample by sample.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <deque>
#include <map>
#include <string>
#include <tuple>
#include <vector>

#include "diagrams.hpp"
#include "device_types.hpp"
#include "kernels.hpp"
#include "mbpt_vegas.h"
#include "runtime.hpp"

using namespace mbpt;

namespace {

constexpr int kMinIters = 3;
constexpr int kMaxPlan = 32;  // iterations per step at most
constexpr int kBlock = 256;
constexpr int kMaxSpt = 16;
constexpr size_t kTermBytesPerSlot = 64 * 1024;
// descriptor entries per slot on average (the largest fourth-order diagram
// group has 22 members)
constexpr int kDiagsPerSlot = 24;
// per-slot iteration-log ring: one step's iterations at most, read back by
// the host after every step
constexpr int kLogIters = kMaxPlan;

size_t a256(size_t x) { return (x + 255) & ~static_cast<size_t>(255); }

// First-fit allocator over [base, base + size) in arbitrary units.
struct Ranges {
  std::map<size_t, size_t> free_;  // start -> length
  void init(size_t base, size_t size) {
    free_.clear();
    if (size) free_[base] = size;
  }
  bool alloc(size_t n, size_t &at) {
    for (auto it = free_.begin(); it != free_.end(); ++it)
      if (it->second >= n) {
        at = it->first;
        const size_t rest = it->second - n;
        free_.erase(it);
        if (rest) free_[at + n] = rest;
        return true;
      }
    return false;
  }
  void release(size_t at, size_t n) {
    if (!n) return;
    auto it = free_.emplace(at, n).first;
    auto nx = std::next(it);
    if (nx != free_.end() && it->first + it->second == nx->first) {
      it->second += nx->second;
      free_.erase(nx);
    }
    if (it != free_.begin()) {
      auto pv = std::prev(it);
      if (pv->first + pv->second == it->first) {
        pv->second += it->second;
        free_.erase(it);
      }
    }
  }
};

// Regularised components of a request and their extrapolation to zero shift
// (index kMaxReg), combined over its iterations on the host: inverse-variance
// sums of the iterations with a positive variance, and count and sum of those
// without (exact: every sample zero or equal).
struct RegSums {
  double w[kMaxReg + 1] = {}, wi[kMaxReg + 1] = {}, zsum[kMaxReg + 1] = {};
  int nzero[kMaxReg + 1] = {};
  int iters = 0;  // iterations folded in
  double E[kMaxReg] = {}, sigma[kMaxReg] = {};
  double E0 = 0.0, sigma0 = 0.0;
  bool ok = false;  // estimates valid (at least one iteration)
};

struct Req {
  mbpt_request r{};
  uint64_t ticket = 0;
  int state = 0;  // 0 queued, 1 resident, 2 done
  int slot = -1;
  double t_submit = 0, t_admit = -1, t_finish = -1;
  mbpt_result res{};
  size_t item_at = 0, item_n = 0, byte_at = 0, byte_n = 0, diag_at = 0, diag_n = 0;
  RegSums reg;
};

struct Layout {
  size_t tasks, olist, diags, grids, hists, reslog, creslog, cache, partials, counters, cpart,
      arena, arena_bytes;
  size_t max_items, max_diags;
};

// Pinned host staging of one step: admitted tables, descriptors and task
// records, the parameter upload, the order list and the state download.  It
// is reused once the step's closing synchronisation has passed.
constexpr size_t kStageBytes = 16u << 20;

// Samples per thread of a server's work items: requests of up to
// max_samples_per_iter samples should still spread over about two blocks per
// CU (a request's iteration latency is that of its slowest block), up to 16.
int server_spt(const mbpt_context *ctx, uint64_t max_samples) {
  const uint64_t per = static_cast<uint64_t>(kBlock) * 2 * std::max(1, ctx->num_cus);
  const uint64_t spt = max_samples / per;
  return static_cast<int>(std::max<uint64_t>(1, std::min<uint64_t>(kMaxSpt, spt)));
}

size_t items_of(uint64_t samples, int spt) {
  const uint64_t chunk = static_cast<uint64_t>(kBlock) * spt;
  return static_cast<size_t>((samples + chunk - 1) / chunk);
}

size_t per_item_bytes(int nreg) {
  return 4 * sizeof(double) + kItemCounters * sizeof(uint64_t) +
         (nreg > 0 ? kRegSums * sizeof(double) : 0);
}

// Slot table, descriptor table, log rings and warm-start cache, then the
// table arena (kTermBytesPerSlot per slot), then the item regions filling the
// rest.  Returns the offset where the item regions begin.
size_t fixed_layout(int slots, int nb, Layout &L) {
  size_t off = 0;
  L.tasks = off;
  off = a256(off + slots * sizeof(TaskDev));
  L.olist = off;
  off = a256(off + slots * sizeof(int2));
  L.diags = off;
  L.max_diags = static_cast<size_t>(slots) * kDiagsPerSlot;
  off = a256(off + L.max_diags * sizeof(DiagDev));
  L.grids = off;
  off = a256(off + static_cast<size_t>(slots) * kMaxDim * (nb + 1) * sizeof(double));
  L.hists = off;
  off = a256(off + static_cast<size_t>(slots) * kMaxDim * nb * sizeof(double));
  L.reslog = off;
  off = a256(off + static_cast<size_t>(slots) * kLogIters * 2 * sizeof(double));
  L.creslog = off;
  off = a256(off + static_cast<size_t>(slots) * kLogIters * kRegSums * sizeof(double));
  L.cache = off;  // grids of recent retirements (warm starts)
  off = a256(off + static_cast<size_t>(slots) * kMaxDim * (nb + 1) * sizeof(double));
  L.arena = off;
  L.arena_bytes = static_cast<size_t>(slots) * kTermBytesPerSlot;
  return off + L.arena_bytes;
}

bool make_layout(int slots, int nb, int nreg, size_t bytes, Layout &L) {
  const size_t off = fixed_layout(slots, nb, L);
  if (bytes <= off + 768) return false;
  const size_t per_item = per_item_bytes(nreg);
  L.max_items = (bytes - off - 768) / per_item;
  if (L.max_items > 0x7fffffffull) L.max_items = 0x7fffffffull;
  L.partials = a256(off);
  L.counters = a256(L.partials + L.max_items * 4 * sizeof(double));
  L.cpart = a256(L.counters + L.max_items * kItemCounters * sizeof(uint64_t));
  const size_t end = nreg > 0 ? L.cpart + L.max_items * kRegSums * sizeof(double) : L.cpart;
  return end <= bytes;
}

double now_s(std::chrono::steady_clock::time_point t0) {
  return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
}

}  // namespace

struct mbpt_server {
  mbpt_context *ctx = nullptr;
  int max_slots = 0, max_queue = 0;
  int spt = 16;  // samples per thread of the work items (server_spt)
  uint64_t max_samples = 0;
  char *ws = nullptr;
  Layout L{};
  Ranges items, bytes, diags;
  int reg_n = 0;          // regularised components of every request (0: none)
  double reg_eta = 0.0;
  std::vector<int64_t> slot_req;  // ticket per slot, -1 if free
  std::vector<TaskDev> h_tasks;
  std::deque<uint64_t> queue;
  std::map<uint64_t, Req> reqs;
  uint64_t next_ticket = 1;
  std::chrono::steady_clock::time_point t0;
  std::vector<FlopModel> flops;
  // compiled descriptors and tables per (order, diagram id or group, group
  // flag), offsets relative to 0
  struct Compiled {
    std::vector<DiagDev> dds;  // one, or the members of a diagram group
    std::vector<GroupDev> groups;
    std::vector<TermDev> terms;
    std::vector<double> coefs;
    FlopModel fm;
    size_t bytes = 0;    // arena bytes of the three tables
    int rc = MBPT_OK;    // compilation status (EINVAL: unknown diagram or group,
                         // label cycle tables that disagree with the label tables)
    std::string err;
  };
  std::map<std::tuple<int, int, int>, Compiled> compiled;
  // pinned staging (see kStageBytes) and its fill level within a step
  char *stage = nullptr;
  size_t stage_used = 0;
  TaskDev *pin_tasks = nullptr;   // parameter upload / state download
  double *pin_creslog = nullptr;  // component log rings (regularised servers)
  int2 *pin_olist = nullptr;
  std::vector<int2> olist;
  std::vector<OrderRange> ranges;
  std::vector<int> admitted;      // slots admitted in the current step
  // warm starts: grids of recent retirements, one cache entry per slot
  struct CacheEntry {
    bool valid = false;
    int order = 0, id = 0, group = 0, matter = 0;
    double density = 0.0, x = 0.0;
    uint64_t stamp = 0;
  };
  std::vector<CacheEntry> cache;
  uint64_t cache_clock = 0, warm_starts = 0;
  double warm_dn = 0.0, warm_dx = 0.0;
  ~mbpt_server() {
    if (ctx) (void)hipStreamSynchronize(ctx->stream);
    if (stage) (void)hipHostFree(stage);
    if (pin_tasks) (void)hipHostFree(pin_tasks);
    if (pin_olist) (void)hipHostFree(pin_olist);
    if (pin_creslog) (void)hipHostFree(pin_creslog);
  }
};

namespace {

KArgs server_kargs(const mbpt_server *s) {
  const mbpt_context *ctx = s->ctx;
  char *b = s->ws;
  KArgs a{};
  a.tasks = reinterpret_cast<TaskDev *>(b + s->L.tasks);
  a.diags = reinterpret_cast<DiagDev *>(b + s->L.diags);
  // group / term offsets of a descriptor are element indices from the
  // workspace base
  a.groups = reinterpret_cast<const GroupDev *>(b);
  a.terms = reinterpret_cast<const TermDev *>(b);
  a.gcoef = reinterpret_cast<const double *>(b);
  a.olist = reinterpret_cast<const int2 *>(b + s->L.olist);
  a.grids = reinterpret_cast<double *>(b + s->L.grids);
  a.hists = reinterpret_cast<double *>(b + s->L.hists);
  a.partials = reinterpret_cast<double *>(b + s->L.partials);
  a.counters = reinterpret_cast<uint64_t *>(b + s->L.counters);
  a.reslog = reinterpret_cast<double *>(b + s->L.reslog);
  a.creslog = reinterpret_cast<double *>(b + s->L.creslog);
  a.cpart = s->reg_n > 0 ? reinterpret_cast<double *>(b + s->L.cpart) : nullptr;
  a.nreg = s->reg_n;
  a.reg_eta = s->reg_eta;
  extrapolation_weights(s->reg_n, a.reg_coef);
  a.ntasks = s->max_slots;
  a.spt = s->spt;
  a.label_mode = ctx->desc.label_mode;
  const mbpt_interaction &v = ctx->v;
  a.phys.V0 = v.C0 * v.hbarc;
  a.phys.Vy = v.Cy * v.hbarc;
  a.phys.m2 = v.mpi * v.mpi;
  a.phys.invLn = std::pow(v.Lambda, -static_cast<double>(v.reg_exp));
  a.phys.hb2m = 0.5 * v.hbar2_m;
  a.phys.half_exp = v.reg_exp / 2;
  a.phys.nb = ctx->desc.n_bins;
  a.phys.seed = ctx->desc.seed;
  a.phys.spectrum = MBPT_SPECTRUM_FREE;
  return a;
}

// Iterations a resident request runs in the next step: the first kMinIters
// at once, then as many as the 1/sqrt(iterations) decrease of the combined
// sigma predicts are needed to reach its target (at least 1, at most
// kMaxPlan), within its evaluation cap.  It depends on the request's own
// state only, so a result does not depend on the requests sharing the GPU.
// With regularised components the estimate is the extrapolation E0 +- sigma0.
int plan_of(const Req &q, bool reg) {
  const mbpt_result &r = q.res;
  const double E = reg ? q.reg.E0 : r.E_per_A, sigma = reg ? q.reg.sigma0 : r.sigma;
  int plan;
  if (r.iters_done < kMinIters || (reg && !q.reg.ok)) {
    plan = std::max(1, kMinIters - r.iters_done);
  } else {
    const double target = std::max(q.r.sigma_rel * std::fabs(E), q.r.sigma_abs);
    if (target > 0.0 && sigma > 0.0) {
      const double ratio = (sigma / target) * (sigma / target);
      const double need = std::ceil(r.iters_done * (ratio - 1.0));
      plan = need < 1.0 ? 1 : (need > kMaxPlan ? kMaxPlan : static_cast<int>(need));
    } else {
      plan = kMaxPlan;
    }
  }
  if (q.r.max_evals > 0) {
    const uint64_t done = r.n_evals, cap = q.r.max_evals, per = q.r.samples_per_iter;
    const uint64_t left = cap > done ? (cap - done + per - 1) / per : 1;
    if (left < static_cast<uint64_t>(plan)) plan = static_cast<int>(std::max<uint64_t>(1, left));
  }
  return plan;
}

// Descriptors and tables of a request's diagram or diagram group, compiled
// once per server (offsets relative to 0).
const mbpt_server::Compiled &compiled_of(mbpt_server *s, int order, int id, int group) {
  auto key = std::make_tuple(order, id, group);
  auto it = s->compiled.find(key);
  if (it != s->compiled.end()) return it->second;
  mbpt_server::Compiled c{};
  mbpt_context *ctx = s->ctx;
  const std::string saved = ctx->err;
  c.rc = compile_task_diagrams(ctx, 4, order, id, group != 0, c.dds, c.groups, c.terms, c.coefs,
                               c.fm);
  if (c.rc) {
    c.err = ctx->err;
    ctx->err = saved;
  }
  c.bytes = a256(c.groups.size() * sizeof(GroupDev)) + a256(c.terms.size() * sizeof(TermDev)) +
            a256(c.coefs.size() * sizeof(double));
  return s->compiled.emplace(key, std::move(c)).first->second;
}

size_t stage_bytes_of(const mbpt_server::Compiled &c) {
  return c.bytes + a256(c.dds.size() * sizeof(DiagDev)) + a256(sizeof(TaskDev));
}

// Returns 0 when admitted, 1 when it does not fit now, < 0 on a HIP error.
int admit_one(mbpt_server *s, Req &q, int slot) {
  mbpt_context *ctx = s->ctx;
  const mbpt_server::Compiled &c = compiled_of(s, q.r.order, q.r.diagram_id, q.r.group);
  const size_t gbytes = a256(c.groups.size() * sizeof(GroupDev));
  const size_t tbytes = a256(c.terms.size() * sizeof(TermDev));
  const size_t need_bytes = c.bytes;
  const size_t need_items = items_of(q.r.samples_per_iter, s->spt);
  const size_t need_diags = c.dds.size();
  const size_t dbytes = a256(need_diags * sizeof(DiagDev));
  // staging: tables (arena image), descriptors, task record
  const size_t stage_need = stage_bytes_of(c);
  if (s->stage_used + stage_need > kStageBytes) return 1;  // next step
  size_t byte_at = 0, item_at = 0, diag_at = 0;
  if (!s->bytes.alloc(need_bytes, byte_at)) return 1;
  if (!s->items.alloc(need_items, item_at)) {
    s->bytes.release(byte_at, need_bytes);
    return 1;
  }
  if (!s->diags.alloc(need_diags, diag_at)) {
    s->bytes.release(byte_at, need_bytes);
    s->items.release(item_at, need_items);
    return 1;
  }
  q.byte_at = byte_at;
  q.byte_n = need_bytes;
  q.item_at = item_at;
  q.item_n = need_items;
  q.diag_at = diag_at;
  q.diag_n = need_diags;
  // byte offsets from the workspace base; the descriptors hold element
  // indices from that base
  const size_t g_off = s->L.arena + byte_at;
  const size_t t_off = g_off + gbytes;
  const size_t c_off = t_off + tbytes;
  const int g_index = static_cast<int>(g_off / sizeof(GroupDev));
  const int t_index = static_cast<int>(t_off / sizeof(TermDev));
  const int c_index = static_cast<int>(c_off / sizeof(double));
  char *st = s->stage + s->stage_used;
  auto *sg = reinterpret_cast<GroupDev *>(st);
  for (size_t i = 0; i < c.groups.size(); ++i) {
    sg[i] = c.groups[i];
    sg[i].first += t_index;
    sg[i].coef_off += c_index;
  }
  std::memcpy(st + gbytes, c.terms.data(), c.terms.size() * sizeof(TermDev));
  std::memcpy(st + gbytes + tbytes, c.coefs.data(), c.coefs.size() * sizeof(double));
  auto *sd = reinterpret_cast<DiagDev *>(st + need_bytes);
  for (size_t i = 0; i < need_diags; ++i) {
    sd[i] = c.dds[i];
    sd[i].group_off += g_index;
    sd[i].term_off += t_index;
  }
  auto *sT = reinterpret_cast<TaskDev *>(st + need_bytes + dbytes);
  TaskDev T{};
  T.diag = static_cast<int>(diag_at);
  T.ndiag = static_cast<int>(need_diags);
  T.nd = 3 * (q.r.order + 1);
  T.grid_off = slot * kMaxDim * (ctx->desc.n_bins + 1);
  T.hist_off = slot * kMaxDim * ctx->desc.n_bins;
  T.res_off = slot * kLogIters;
  T.res_cap = kLogIters;
  T.key = static_cast<uint32_t>(q.ticket);
  T.order = q.r.order;
  T.nsamples = q.r.samples_per_iter;
  T.nitems = static_cast<int>(need_items);
  T.store_begin = static_cast<int>(item_at);
  const double x = q.r.matter == MBPT_NUCLEAR ? q.r.proton_fraction : 0.0;
  fill_medium(ctx, q.r.density, x, T);
  T.active = 1;
  s->h_tasks[slot] = T;
  *sT = T;
  char *b = s->ws;
  // asynchronous copies from pinned staging: the step's closing
  // synchronisation orders them before the staging is reused
  if (need_bytes)
    MBPT_HIPCHK(ctx, hipMemcpyAsync(b + g_off, st, need_bytes, hipMemcpyHostToDevice, ctx->stream));
  MBPT_HIPCHK(ctx, hipMemcpyAsync(b + s->L.diags + diag_at * sizeof(DiagDev), sd,
                                  need_diags * sizeof(DiagDev), hipMemcpyHostToDevice,
                                  ctx->stream));
  MBPT_HIPCHK(ctx, hipMemcpyAsync(b + s->L.tasks + slot * sizeof(TaskDev), sT, sizeof(TaskDev),
                                  hipMemcpyHostToDevice, ctx->stream));
  KArgs a = server_kargs(s);
  MBPT_HIPCHK(ctx, launch_init(a, slot, 1, ctx->stream));
  if (s->warm_dn > 0.0) {
    // nearest retired grid of the same diagram and matter within the window
    int best = -1;
    double best_d = 0.0;
    const int matter = q.r.matter;
    for (int e = 0; e < static_cast<int>(s->cache.size()); ++e) {
      const auto &ce = s->cache[e];
      if (!ce.valid || ce.order != q.r.order || ce.id != q.r.diagram_id ||
          ce.group != q.r.group || ce.matter != matter)
        continue;
      const double dn = std::fabs(ce.density - q.r.density), dx = std::fabs(ce.x - q.r.proton_fraction);
      if (dn > s->warm_dn || dx > s->warm_dx) continue;
      const double dist = dn / s->warm_dn + (s->warm_dx > 0.0 ? dx / s->warm_dx : 0.0);
      if (best < 0 || dist < best_d) {
        best = e;
        best_d = dist;
      }
    }
    if (best >= 0) {
      const size_t gbytes = static_cast<size_t>(T.nd) * (ctx->desc.n_bins + 1) * sizeof(double);
      MBPT_HIPCHK(ctx, hipMemcpyAsync(b + s->L.grids + T.grid_off * sizeof(double),
                                      b + s->L.cache + best * kMaxDim * (ctx->desc.n_bins + 1) *
                                                           sizeof(double),
                                      gbytes, hipMemcpyDeviceToDevice, ctx->stream));
      s->cache[best].stamp = ++s->cache_clock;
      ++s->warm_starts;
    }
  }
  s->stage_used += stage_need;
  s->flops[slot] = c.fm;
  q.state = 1;
  q.slot = slot;
  q.t_admit = now_s(s->t0);
  s->slot_req[slot] = static_cast<int64_t>(q.ticket);
  return 0;
}

// Folds the iterations a request ran since the last step into its sums of
// the components and of the extrapolation (from the slot's log ring, read back
// with the step's state: components in the first pairs of a log entry, the
// extrapolation in its last pair) and updates the estimates: each combines its
// iterations by inverse variance; iterations without variance are exact
// (their plain mean, sigma 0, as for the main estimate).
void fold_components(mbpt_server *s, Req &q, const TaskDev &S) {
  RegSums &g = q.reg;
  const int K = s->reg_n;
  for (int it = g.iters; it < S.it_done; ++it) {
    const double *cl = s->pin_creslog + static_cast<size_t>(S.res_off + it % kLogIters) * kRegSums;
    for (int j = 0; j <= K; ++j) {
      const int r = j < K ? j : kMaxReg;
      const double I = cl[2 * r], v = cl[2 * r + 1];
      if (v > 0.0) {
        g.w[r] += 1.0 / v;
        g.wi[r] += I / v;
      } else {
        g.zsum[r] += I;
        ++g.nzero[r];
      }
    }
  }
  g.iters = S.it_done;
  if (g.iters < 1) return;
  for (int j = 0; j <= K; ++j) {
    const int r = j < K ? j : kMaxReg;
    const double E = g.nzero[r] > 0 ? g.zsum[r] / g.nzero[r] : g.wi[r] / g.w[r];
    const double sg = g.nzero[r] > 0 ? 0.0 : 1.0 / std::sqrt(g.w[r]);
    if (j < K) {
      g.E[j] = E;
      g.sigma[j] = sg;
    } else {
      g.E0 = E;
      g.sigma0 = sg;
    }
  }
  g.ok = true;
}

}  // namespace

extern "C" int mbpt_server_workspace_query(const mbpt_context *ctx, int max_slots,
                                           uint64_t max_samples_per_iter, size_t *bytes) {
  if (!ctx || !bytes || max_slots < 1 || max_samples_per_iter < 2) return MBPT_EINVAL;
  Layout L{};
  *bytes = fixed_layout(max_slots, ctx->desc.n_bins, L) +
           static_cast<size_t>(max_slots) *
               items_of(max_samples_per_iter, server_spt(ctx, max_samples_per_iter)) *
               per_item_bytes(ctx->reg_n) +
           2048;
  return MBPT_OK;
}

extern "C" int mbpt_server_create(mbpt_context *ctx, int max_slots, uint64_t max_samples_per_iter,
                                  int max_queue, void *device_ptr, size_t bytes,
                                  mbpt_server **out) {
  if (!ctx || !out || max_slots < 1 || max_samples_per_iter < 2 || max_queue < 1 || !device_ptr ||
      (reinterpret_cast<uintptr_t>(device_ptr) & 255u))
    return MBPT_EINVAL;
  *out = nullptr;
  if (ctx->desc.spectrum != MBPT_SPECTRUM_FREE) {
    set_err(ctx, "server_create: the server supports the free spectrum only");
    return MBPT_EINVAL;
  }
  if (!fixed_masks_ok()) {
    set_err(ctx, "internal: the generator's descriptors differ from the kernels' compile-time "
                 "tables or exceed their group limit");
    return MBPT_EINVAL;
  }
  Layout L{};
  if (!make_layout(max_slots, ctx->desc.n_bins, ctx->reg_n, bytes, L) ||
      L.max_items < items_of(max_samples_per_iter, server_spt(ctx, max_samples_per_iter))) {
    set_err(ctx, "server_create: workspace too small for the slot table and one request");
    return MBPT_ENOMEM;
  }
  auto *s = new mbpt_server();
  s->ctx = ctx;
  s->max_slots = max_slots;
  s->max_queue = max_queue;
  s->max_samples = max_samples_per_iter;
  s->spt = server_spt(ctx, max_samples_per_iter);
  s->ws = static_cast<char *>(device_ptr);
  s->L = L;
  s->items.init(0, L.max_items);
  s->bytes.init(0, L.arena_bytes);
  s->diags.init(0, L.max_diags);
  s->reg_n = ctx->reg_n;
  s->reg_eta = ctx->reg_eta;
  s->slot_req.assign(max_slots, -1);
  s->cache.assign(max_slots, mbpt_server::CacheEntry{});
  s->h_tasks.assign(max_slots, TaskDev{});
  s->flops.assign(max_slots, FlopModel{});
  s->t0 = std::chrono::steady_clock::now();
  if (hipHostMalloc(reinterpret_cast<void **>(&s->stage), kStageBytes, hipHostMallocDefault) !=
          hipSuccess ||
      hipHostMalloc(reinterpret_cast<void **>(&s->pin_tasks), max_slots * sizeof(TaskDev),
                    hipHostMallocDefault) != hipSuccess ||
      hipHostMalloc(reinterpret_cast<void **>(&s->pin_olist), max_slots * sizeof(int2),
                    hipHostMallocDefault) != hipSuccess ||
      (s->reg_n > 0 &&
       hipHostMalloc(reinterpret_cast<void **>(&s->pin_creslog),
                     static_cast<size_t>(max_slots) * kLogIters * kRegSums * sizeof(double),
                     hipHostMallocDefault) != hipSuccess)) {
    set_err(ctx, "server_create: pinned host allocation failed");
    delete s;
    return MBPT_EHIP;
  }
  std::memset(s->pin_tasks, 0, max_slots * sizeof(TaskDev));
  if (hipMemcpyAsync(s->ws + L.tasks, s->pin_tasks, max_slots * sizeof(TaskDev),
                     hipMemcpyHostToDevice, ctx->stream) != hipSuccess ||
      hipStreamSynchronize(ctx->stream) != hipSuccess) {
    set_err(ctx, "server_create: HIP copy failed");
    delete s;
    return MBPT_EHIP;
  }
  *out = s;
  return MBPT_OK;
}

extern "C" void mbpt_server_destroy(mbpt_server *s) { delete s; }

extern "C" int mbpt_server_submit(mbpt_server *s, const mbpt_request *req, uint64_t *ticket) {
  if (!s || !req || !ticket) return MBPT_EINVAL;
  mbpt_context *ctx = s->ctx;
  const bool known = req->group == 1 ? !group_members(req->order, req->diagram_id).empty()
                                       : req->group == 0 && get_diagram(req->order, req->diagram_id);
  if (!known || !(req->density > 0) || !(req->proton_fraction >= 0 && req->proton_fraction <= 1) ||
      (req->matter != MBPT_NEUTRON && req->matter != MBPT_NUCLEAR) ||
      (req->matter == MBPT_NEUTRON && req->proton_fraction != 0.0) || req->samples_per_iter < 2 ||
      req->samples_per_iter > s->max_samples || !(req->sigma_rel >= 0) || !(req->sigma_abs >= 0)) {
    set_err(ctx, "server_submit: invalid request");
    return MBPT_EINVAL;
  }
  if (static_cast<int>(s->queue.size()) >= s->max_queue) {
    set_err(ctx, "server_submit: queue full");
    return MBPT_EBUSY;
  }
  const mbpt_server::Compiled &c = compiled_of(s, req->order, req->diagram_id, req->group);
  if (c.rc) {
    set_err(ctx, "server_submit: " + c.err);
    return c.rc;
  }
  // a request that could never be admitted, even into an empty server
  if (c.bytes > s->L.arena_bytes || c.dds.size() > s->L.max_diags ||
      stage_bytes_of(c) > kStageBytes) {
    set_err(ctx, "server_submit: the request's " + std::to_string(c.dds.size()) +
                     " descriptors and " + std::to_string(c.bytes) +
                     " table bytes exceed the server's descriptor table (" +
                     std::to_string(s->L.max_diags) + ") or table arena (" +
                     std::to_string(s->L.arena_bytes) + " bytes)");
    return MBPT_ENOMEM;
  }
  Req q;
  q.r = *req;
  q.ticket = s->next_ticket++;
  q.t_submit = now_s(s->t0);
  s->reqs[q.ticket] = q;
  s->queue.push_back(q.ticket);
  *ticket = q.ticket;
  return MBPT_OK;
}

extern "C" int mbpt_server_step(mbpt_server *s, int *n_active, int *n_queued) {
  if (!s) return MBPT_EINVAL;
  mbpt_context *ctx = s->ctx;
  if (ctx->desc.spectrum != MBPT_SPECTRUM_FREE) {
    set_err(ctx, "server_step: the server supports the free spectrum only");
    return MBPT_ESTATE;
  }
  const bool reg = s->reg_n > 0;
  while (!s->queue.empty()) {
    int slot = -1;
    for (int i = 0; i < s->max_slots; ++i)
      if (s->slot_req[i] < 0) {
        slot = i;
        break;
      }
    if (slot < 0) break;
    Req &q = s->reqs[s->queue.front()];
    const int rc = admit_one(s, q, slot);
    if (rc == 1) break;  // no room: wait for retirements
    if (rc < 0) return rc;
    s->queue.pop_front();
  }
  // plans, and work numbering grouped by order over the resident slots (free
  // slots own none), longest plan first within an order: in iteration j of
  // the step the requests still running are a prefix of each order's list
  std::vector<int> active;
  int K = 0;
  for (int i = 0; i < s->max_slots; ++i) {
    TaskDev &T = s->h_tasks[i];
    if (s->slot_req[i] >= 0) {
      T.plan = plan_of(s->reqs[static_cast<uint64_t>(s->slot_req[i])], reg);
      K = std::max(K, T.plan);
      active.push_back(i);
    } else {
      T.nitems = 0;
      T.active = 0;
      T.plan = 0;
    }
  }
  std::stable_sort(active.begin(), active.end(), [&](int x, int y) {
    return s->h_tasks[x].plan > s->h_tasks[y].plan;
  });
  const int nactive = static_cast<int>(active.size());
  if (nactive > 0) {
    order_items(s->h_tasks, active, s->olist, s->ranges);
    std::memcpy(s->pin_tasks, s->h_tasks.data(), s->max_slots * sizeof(TaskDev));
    std::memcpy(s->pin_olist, s->olist.data(), s->olist.size() * sizeof(int2));
    const size_t width = offsetof(TaskDev, iter);
    MBPT_HIPCHK(ctx, hipMemcpy2DAsync(s->ws + s->L.tasks, sizeof(TaskDev), s->pin_tasks,
                                      sizeof(TaskDev), width, s->max_slots, hipMemcpyHostToDevice,
                                      ctx->stream));
    MBPT_HIPCHK(ctx, hipMemcpyAsync(s->ws + s->L.olist, s->pin_olist,
                                    s->olist.size() * sizeof(int2), hipMemcpyHostToDevice,
                                    ctx->stream));
    KArgs a = server_kargs(s);
    a.total_items = s->ranges.back().item_end;
    const int prec = ctx->desc.precision;
    size_t slot = 0;
    timed_begin(ctx, slot);
    for (int j = 0; j < K; ++j) {
      for (const auto &r : s->ranges) {
        int k1 = r.k0;  // end of the prefix still running in iteration j
        while (k1 < r.k1 && s->h_tasks[s->olist[k1].y].plan > j) ++k1;
        if (k1 == r.k0) continue;
        const int end = k1 < r.k1 ? s->olist[k1].x : r.item_end;
        MBPT_HIPCHK(ctx, launch_sample_order(a, r.order, 4, prec, r.group, r.k0, k1,
                                             end - s->olist[r.k0].x, kBlock, ctx->stream));
      }
      MBPT_HIPCHK(ctx, launch_finish(a, 0, s->max_slots, j, ctx->desc.alpha, ctx->stream));
    }
    timed_end(ctx, slot);
    const TaskDev *st = s->pin_tasks;
    MBPT_HIPCHK(ctx, hipMemcpyAsync(s->pin_tasks, s->ws + s->L.tasks,
                                    s->max_slots * sizeof(TaskDev), hipMemcpyDeviceToHost,
                                    ctx->stream));
    if (reg)
      MBPT_HIPCHK(ctx, hipMemcpyAsync(s->pin_creslog, s->ws + s->L.creslog,
                                      static_cast<size_t>(s->max_slots) * kLogIters * kRegSums *
                                          sizeof(double),
                                      hipMemcpyDeviceToHost, ctx->stream));
    MBPT_HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
    s->stage_used = 0;
    resolve_timing(ctx);
    const double t = now_s(s->t0);
    uint64_t evals = 0;
    double flops = 0.0;
    for (int i = 0; i < s->max_slots; ++i) {
      if (s->slot_req[i] < 0) continue;
      Req &q = s->reqs[static_cast<uint64_t>(s->slot_req[i])];
      const TaskDev &S = st[i];
      TaskDev &H = s->h_tasks[i];  // host copy keeps last round's counters
      evals += S.nevals - H.nevals;
      flops += s->flops[i].pre * (S.nevals - H.nevals) + s->flops[i].post * (S.npass - H.npass) +
               s->flops[i].per_term * (S.nterms - H.nterms);
      H.nevals = S.nevals;
      H.npass = S.npass;
      H.nterms = S.nterms;
      result_of(S, q.res);
      if (reg) fold_components(s, q, S);
      const double E = reg ? q.reg.E0 : q.res.E_per_A, sigma = reg ? q.reg.sigma0 : q.res.sigma;
      const double target = std::max(q.r.sigma_rel * std::fabs(E), q.r.sigma_abs);
      const bool converged =
          S.it_done >= kMinIters && sigma <= target && (!reg || q.reg.ok);
      const bool capped = q.r.max_evals > 0 && S.nevals >= q.r.max_evals;
      if (converged || capped || !std::isfinite(q.res.E_per_A) || (reg && !std::isfinite(E))) {
        q.state = 2;
        q.t_finish = t;
        if (s->warm_dn > 0.0 && S.it_done >= kMinIters && std::isfinite(q.res.E_per_A)) {
          // keep the adapted grid: replace the least recently used entry
          int e = 0;
          for (int k = 1; k < static_cast<int>(s->cache.size()); ++k)
            if (!s->cache[k].valid || (s->cache[e].valid && s->cache[k].stamp < s->cache[e].stamp))
              e = k;
          auto &ce = s->cache[e];
          ce.valid = true;
          ce.order = q.r.order;
          ce.id = q.r.diagram_id;
          ce.group = q.r.group;
          ce.matter = q.r.matter;
          ce.density = q.r.density;
          ce.x = q.r.proton_fraction;
          ce.stamp = ++s->cache_clock;
          const size_t gbytes = static_cast<size_t>(S.nd) * (ctx->desc.n_bins + 1) * sizeof(double);
          MBPT_HIPCHK(ctx, hipMemcpyAsync(
                               s->ws + s->L.cache + e * kMaxDim * (ctx->desc.n_bins + 1) * sizeof(double),
                               s->ws + s->L.grids + S.grid_off * sizeof(double), gbytes,
                               hipMemcpyDeviceToDevice, ctx->stream));
        }
        s->bytes.release(q.byte_at, q.byte_n);
        s->items.release(q.item_at, q.item_n);
        s->diags.release(q.diag_at, q.diag_n);
        s->slot_req[i] = -1;
        H = TaskDev{};
      }
    }
    ctx->evals += evals;
    ctx->flops += flops;
  }
  int na = 0;
  for (int i = 0; i < s->max_slots; ++i) na += s->slot_req[i] >= 0;
  if (n_active) *n_active = na;
  if (n_queued) *n_queued = static_cast<int>(s->queue.size());
  return MBPT_OK;
}

extern "C" int mbpt_server_set_warm_start(mbpt_server *s, double max_dn, double max_dx) {
  if (!s || !(max_dx >= 0.0) || std::isnan(max_dn)) return MBPT_EINVAL;
  s->warm_dn = max_dn > 0.0 ? max_dn : 0.0;
  s->warm_dx = max_dx;
  return MBPT_OK;
}

extern "C" int mbpt_server_warm_starts(const mbpt_server *s, uint64_t *count) {
  if (!s || !count) return MBPT_EINVAL;
  *count = s->warm_starts;
  return MBPT_OK;
}

extern "C" int mbpt_server_poll(mbpt_server *s, uint64_t ticket, mbpt_result *res, int *done,
                                double *t_submit, double *t_admit, double *t_finish) {
  if (!s) return MBPT_EINVAL;
  auto it = s->reqs.find(ticket);
  if (it == s->reqs.end()) return MBPT_EINVAL;
  const Req &q = it->second;
  if (res) *res = q.res;
  if (done) *done = q.state == 2;
  if (t_submit) *t_submit = q.t_submit;
  if (t_admit) *t_admit = q.t_admit;
  if (t_finish) *t_finish = q.t_finish;
  return MBPT_OK;
}

extern "C" int mbpt_server_poll_regularized(mbpt_server *s, uint64_t ticket, double *E,
                                            double *sigma, double *E0, double *sigma0) {
  if (!s) return MBPT_EINVAL;
  auto it = s->reqs.find(ticket);
  if (it == s->reqs.end()) return MBPT_EINVAL;
  const Req &q = it->second;
  if (s->reg_n < 1 || q.reg.iters < 1 || !q.reg.ok) {
    set_err(s->ctx, s->reg_n < 1 ? "server_poll_regularized: the server has no regularised "
                                   "components"
                                 : "server_poll_regularized: no iteration yet");
    return MBPT_ESTATE;
  }
  for (int k = 0; k < s->reg_n; ++k) {
    if (E) E[k] = q.reg.E[k];
    if (sigma) sigma[k] = q.reg.sigma[k];
  }
  if (E0) *E0 = q.reg.E0;
  if (sigma0) *sigma0 = q.reg.sigma0;
  return MBPT_OK;
}
