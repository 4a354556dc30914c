// Handle types behind the opaque C ABI pointers.
#pragma once
#include <hip/hip_runtime.h>

#include <string>
#include <utility>
#include <vector>

#include "device_types.hpp"
#include "mbpt_vegas.h"

namespace mbpt {

// One sample launch over the tasks of one order: olist entries [k0, k1),
// nitems items ending at item_end.
struct OrderRange {
  int order, k0, k1, item_end, nitems;
  bool group;  // some task of the range is a diagram group
};

// Algorithmic FLOPs of one evaluation (see count_flops).
struct FlopModel {
  double pre = 0.0;        // every sample
  double post = 0.0;       // samples past the Pauli test
  double per_term = 0.0;   // per label unit evaluated (isospin group or explicit term)
  double transc_pre = 0.0, transc_post = 0.0;
  double all_units = 0.0;  // label units of the whole list (groups or terms)
  double shared = 0.0, transc_shared = 0.0;  // part of pre a diagram group pays once
};

}  // namespace mbpt

struct mbpt_context {
  mbpt_context_desc desc{};
  hipStream_t stream = nullptr;
  mbpt_interaction v{};
  int num_cus = 256;
  std::string err;
  std::vector<std::pair<hipEvent_t, hipEvent_t>> events;
  size_t n_used = 0;
  uint64_t launches = 0;
  double kernel_ms = 0.0;
  uint64_t evals = 0;
  double flops = 0.0;
  uint64_t epoch = 0;  // bumped when precision or interaction changes
  int reg_n = 0;         // regularised components (0: none)
  double reg_eta = 0.0;  // component k shifts every denominator by -k reg_eta
  double fp32_rel_target = 0.0;  // see mbpt_set_fp32_target
};

struct mbpt_task_set {
  mbpt_context *ctx = nullptr;
  uint64_t epoch = ~uint64_t{0};  // context epoch the launches were set up for
  int q = 2;
  std::vector<mbpt_task_desc> tasks;
  int launch_mode = MBPT_LAUNCH_PER_TASK;
  int train_iters = 0;  // training/evaluation split (0: off)
  int block = 256, spt = 16;
  bool blocking_auto = true;  // spt chosen at bind from the sample count
  std::vector<mbpt::DiagDev> diags;
  std::vector<mbpt::GroupDev> groups;
  std::vector<mbpt::TermDev> terms;
  std::vector<double> coefs;        // see coef_slots
  std::vector<int> task_diag, task_ndiag;  // first descriptor and count per task
  std::vector<mbpt::FlopModel> flops;
  int max_nd = 0;
  std::vector<mbpt::TaskDev> h_tasks, last_state;
  int grid_doubles = 0, hist_doubles = 0;
  // workspace
  char *ws = nullptr;
  size_t ws_bytes = 0;
  uint64_t max_samples = 0;
  int max_iters = 0;
  size_t max_items = 0;
  mbpt::TaskDev *d_tasks = nullptr;
  int2 *d_olist = nullptr;
  mbpt::DiagDev *d_diags = nullptr;
  mbpt::GroupDev *d_groups = nullptr;
  mbpt::TermDev *d_terms = nullptr;
  double *d_coefs = nullptr;
  double *d_hf = nullptr;   // HF spline entries (2 tables per task)
  double *d_gl = nullptr;   // Gauss-Legendre rule for the HF tables
  bool hf_dirty = true;     // HF tables must be (re)computed before use
  std::vector<double> h_gl; // host copy of the rule (source of an async copy)
  double *d_grids = nullptr, *d_hists = nullptr, *d_partials = nullptr, *d_reslog = nullptr;
  double *d_cpart = nullptr, *d_creslog = nullptr;  // regularised components
  // regularisation the logged iterations ran with (fixed from the first
  // iteration after a reset)
  int run_reg_n = -1;
  double run_reg_eta = 0.0;
  uint64_t *d_counters = nullptr;
  int *d_queue = nullptr;  // work-item counters of the persistent launches
  std::vector<int2> olist;                 // (first item, task) grouped by order
  std::vector<mbpt::OrderRange> oranges;   // one sample launch per order
  hipGraphExec_t graph_exec = nullptr;
  int graph_iters = 0;
  // set while mbpt_integrate_noalloc runs: no graph capture, no timing events
  bool noalloc = false;
  void drop_graph() {
    if (graph_exec) (void)hipGraphExecDestroy(graph_exec);
    graph_exec = nullptr;
    graph_iters = 0;
  }
};

namespace mbpt {
struct Diagram;
void set_err(mbpt_context *ctx, const std::string &msg);
int hip_fail(mbpt_context *ctx, hipError_t e, const char *what);
void count_flops(const Diagram &d, int q, int half_exp, int label_mode, int spectrum,
                 FlopModel &f);
bool append_label_tables(const Diagram &d, int q, DiagDev &dd, std::vector<GroupDev> &groups,
                         std::vector<TermDev> &terms, std::vector<double> &coefs,
                         size_t group_base, size_t term_base, size_t coef_base,
                         bool canonical = false);
void fill_diag_dev(const Diagram &d, DiagDev &dd, bool canonical = false);
// Descriptors (appended to dds), label tables (appended to groups, terms,
// coefs; a descriptor's offsets index those vectors) and the combined FLOP
// model of one task: one diagram, or with group the members of the order's
// diagram group with id particle-carried loops, in canonical loop order.
int compile_task_diagrams(mbpt_context *ctx, int q, int order, int id, bool group,
                          std::vector<DiagDev> &dds, std::vector<GroupDev> &groups,
                          std::vector<TermDev> &terms, std::vector<double> &coefs,
                          FlopModel &model);
bool poly_fit_at_zero(const double *x, const double *y, const double *sig, int n, int deg,
                      double &c0, double &s0);
void extrapolation_weights(int K, double *a);
bool fixed_masks_ok();
void fill_medium(const mbpt_context *ctx, double density, double x, TaskDev &T);
void result_of(const TaskDev &S, mbpt_result &r);
void timed_begin(mbpt_context *ctx, size_t &slot);
void timed_end(mbpt_context *ctx, size_t slot);
void resolve_timing(mbpt_context *ctx);
void gauss_legendre(int n, double *x, double *w);
int ensure_hf(mbpt_task_set *set);
int sync_epoch(mbpt_task_set *set);
void order_items(std::vector<TaskDev> &T, const std::vector<int> &active,
                 std::vector<int2> &olist, std::vector<OrderRange> &ranges);
int integrate_in(mbpt_task_set *set, void *base, size_t bytes, uint64_t samples_per_iter,
                 int iters, mbpt_result *per_task, mbpt_result *total);
}  // namespace mbpt

#define MBPT_HIPCHK(ctx, call)                                      \
  do {                                                              \
    hipError_t e_ = (call);                                         \
    if (e_ != hipSuccess) return ::mbpt::hip_fail(ctx, e_, #call);  \
  } while (0)
