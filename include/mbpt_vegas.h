/*
 * mbpt_vegas.h -- C ABI of the MI355X (gfx950) VEGAS Monte Carlo library for
 * many-body perturbation theory (MBPT) energy diagrams of infinite nucleon
 * matter (arXiv:2603.24532, Secs. "Many-body expressions" and "Automated
 * evaluation of many-body expressions").
 *
 * What is computed.  For a two-body Hugenholtz energy diagram of order n at an
 * equation-of-state point (total density n_B, proton fraction x), the library
 * estimates the diagram's contribution to the energy per particle E/A [MeV],
 * i.e. the momentum integral of Eqs. (1)-(5) generalised to order n (sum over
 * holes and particles with n_k, 1 - n_k Pauli factors, antisymmetrised
 * matrix elements with explicit spin(-isospin) sums, energy denominators of
 * eq:Dijkabc with a free spectrum) divided by n_B, by adaptive importance
 * sampling on a per-dimension piecewise-linear grid (VEGAS, Sec. "MC
 * integration": training with refinement, inverse-variance combination).
 *
 * Conventions for every entry point:
 *  - Return value: MBPT_OK (0) or a negative MBPT_E* code; no C++ exception
 *    crosses the ABI.  After an error, mbpt_last_error(ctx) describes it.
 *  - Handles are opaque and owned by the library; destroy them with the
 *    matching *_destroy call.  A context and everything created from it are
 *    used from one host thread at a time.
 *  - Device memory is never allocated by the library: the caller binds a
 *    device workspace (for instance a PyTorch uint8 tensor) whose size it gets
 *    from mbpt_workspace_query; the library keeps the pointer until unbound or
 *    destroyed and never frees it.  All GPU work is queued on the HIP stream
 *    given at context creation (for instance torch.cuda.current_stream()).
 *  - Host pointers are read (inputs) or written (outputs) only during the call.
 */
#ifndef MBPT_VEGAS_H
#define MBPT_VEGAS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- status codes ---------------------------------------------------- */
#define MBPT_OK 0
#define MBPT_EINVAL (-1)   /* invalid argument                              */
#define MBPT_ENOMEM (-2)   /* bound workspace too small for the request     */
#define MBPT_EHIP (-3)     /* a HIP runtime call failed (message retained)   */
#define MBPT_ENUMERIC (-4) /* non-finite estimate                            */
#define MBPT_EBUSY (-5)    /* server queue full                              */
#define MBPT_ESTATE (-6)   /* call not valid in the current state            */

/* ---- enums ------------------------------------------------------------ */
/* Integrand arithmetic.  FP64: everything in double.  FP32: the per-sample
 * integrand in float with the variance sums, the grid refinement and every
 * sample inside the near-Fermi-surface / small-denominator band re-evaluated in
 * double (fp64 accumulation, compensated across threads and work items). */
enum { MBPT_FP64 = 0, MBPT_FP32 = 1 };
/* Matter: NEUTRON = pure neutron matter, spin labels only (degeneracy 2,
 * proton fraction must be 0); NUCLEAR = spin x isospin labels (degeneracy 4),
 * isospin-dependent Pauli factors, any proton fraction in [0, 1]. */
enum { MBPT_NEUTRON = 0, MBPT_NUCLEAR = 1 };
/* How mbpt_integrate launches work.  PER_TASK: one sample launch per task and
 * iteration (the plain path; within an iteration the tasks in turn, then one
 * iteration-end launch for all of them); BATCHED: per iteration one sample launch
 * per order present, each covering the work items of every task of that order
 * (one block per work item), then one iteration-end launch; GRAPH: BATCHED with the whole iteration
 * sequence captured once into a HIP graph and replayed (needs a non-default
 * stream: EINVAL on the null stream); PERSISTENT: per iteration one
 * persistent launch per order present (about as many blocks as are resident
 * at once; each claims chunks of work items from a counter, keeps the current
 * task's grid and histogram in LDS across its items and merges the histogram
 * once per run of a task's items), then the iteration-end launch. */
enum {
  MBPT_LAUNCH_PER_TASK = 0,
  MBPT_LAUNCH_BATCHED = 1,
  MBPT_LAUNCH_GRAPH = 2,
  MBPT_LAUNCH_PERSISTENT = 3
};
/* Single-particle energies in the energy denominators (eq:Dijkabc).  FREE:
 * eps = hbar^2 k^2 / 2m.  HF: the Hartree-Fock spectrum of eq:spe,
 * eps_tau(k) = hbar^2 k^2 / 2m + Sigma_tau(k) with Sigma_tau(k) the sum over
 * occupied partners of <k tau, j|V(1 - P12)|k tau, j>; isospin dependent in
 * asymmetric matter (the paper's explicit treatment, no isospin averaging).
 * Sigma is tabulated per task once per medium on 512 equal steps of
 * [0, kF,max + 6 Lambda] by 64 x 64-point Gauss-Legendre quadrature and
 * interpolated by a cubic spline with zero end slopes (the paper's fine grid
 * plus cubic spline, Sec. "Automated evaluation").  The FP32 integrand
 * implements FREE only: with HF every sample takes the fp64 path.  The
 * continuous-batching server supports FREE only. */
enum { MBPT_SPECTRUM_FREE = 0, MBPT_SPECTRUM_HF = 1 };

/* ---- value types -------------------------------------------------------- */
/* Two-body interaction V(p,p') = hbarc [C0 + Cy/(|p-p'|^2 + mpi^2)]
 * exp(-(p/Lambda)^reg_exp) exp(-(p'/Lambda)^reg_exp), antisymmetrised as
 * <12|V(1 - P12)|34> (Sec. "Implementing chiral forces": regulator f_NN of the
 * nonlocal form, commuting with the antisymmetrizer).  Units: C0 [fm^2], Cy
 * dimensionless, mpi and Lambda [fm^-1], hbar2_m = hbar^2/m [MeV fm^2], hbarc
 * [MeV fm].  reg_exp must be an even integer in [2, 16]; reg_exp = 4 runs
 * sample kernels with the exponent fixed at compile time (the fastest), other
 * values run kernels that read it at launch (the same operations). */
typedef struct mbpt_interaction {
  double C0, Cy, mpi, Lambda;
  int reg_exp;
  double hbar2_m, hbarc;
} mbpt_interaction;

/* Context creation parameters.  stream: a hipStream_t (NULL = default
 * stream).  n_bins: VEGAS bins per dimension (2..128).  alpha: refinement
 * exponent.  kcut_extra: particle-line loop momenta are sampled in a ball of
 * radius kF,max + kcut_extra * Lambda (hole lines: kF,max, exact).
 * fp32_band_k, fp32_band_d: FP32 precision only -- a sample is re-evaluated
 * in fp64 if some line has |k^2 - kF^2| < band_k kF^2 or some denominator has
 * |D| < band_d * (sum of |eps| over its lines).  label_mode: 0 evaluates the
 * spin(-isospin) sum of each isospin configuration as its multilinear
 * polynomial in the vertex matrix elements (coefficients compiled from the
 * nonzero label assignments); 1 evaluates the compressed list of nonzero
 * assignments term by term.  Both are exact; 0 is faster at high orders. */
typedef struct mbpt_context_desc {
  int device;
  void *stream;
  int precision;
  uint32_t seed;
  int n_bins;
  double alpha;
  double kcut_extra;
  double fp32_band_k;
  double fp32_band_d;
  int label_mode;
  int spectrum;
} mbpt_context_desc;

/* One integration task: diagram `diagram_id` of order `order` (1..5; ids
 * index the deterministic generator list, see mbpt_num_diagrams) at density
 * [fm^-3] and proton fraction.  task_key is the second Philox key word: the
 * random stream of a task is (seed, task_key, iteration, sample).
 * group = 1: the task is a diagram group (Sec. "Automated evaluation": sums
 * of diagrams of one order and particle-hole composition integrated
 * together): diagram_id is then the number p of loop momenta carried by
 * particle lines, and the task integrates the sum of the integrands of the
 * order's diagrams with that p (mbpt_group_members), each member's loops
 * taken particle loops first so that all share the loop radii; one VEGAS
 * grid adapts to the sum.  Free spectrum only.  group = 0: one diagram. */
typedef struct mbpt_task_desc {
  int order;
  int diagram_id;
  int matter;
  double density;
  double proton_fraction;
  uint32_t task_key;
  int group;
} mbpt_task_desc;

/* Result of one task (or a sum over tasks).  E_per_A: inverse-variance
 * weighted mean over all iterations run so far [MeV]; sigma its standard
 * error; chi2_dof the consistency of the iterations; last_E/last_sigma the
 * last iteration alone; n_evals integrand evaluations; n_fp64_fallback samples
 * re-evaluated in fp64 (FP32 precision). */
typedef struct mbpt_result {
  double E_per_A, sigma, chi2_dof, last_E, last_sigma;
  int iters_done;
  uint64_t n_evals;
  uint64_t n_fp64_fallback;
} mbpt_result;

typedef struct mbpt_context mbpt_context;
typedef struct mbpt_task_set mbpt_task_set;
typedef struct mbpt_server mbpt_server;

/* ---- context -------------------------------------------------------------- */
/* Create a context on `device`.  desc may be NULL for defaults (device 0,
 * default stream, FP64, seed 1, 50 bins, alpha 1.5, kcut_extra 3.0, bands
 * 1e-4 / 1e-2, label_mode 0, spectrum FREE).  The default interaction is the synthetic contact + Yukawa one
 * (C0 = -1 fm^2, Cy = -2, mpi = 0.7, Lambda = 2, exponent 4, hbar^2/m = 41.47,
 * hbarc = 197.3269804).  EINVAL on bad fields, EHIP if the device is absent. */
int mbpt_context_create(const mbpt_context_desc *desc, mbpt_context **out);
void mbpt_context_destroy(mbpt_context *ctx);
/* Message of the last failed call on this context (never NULL). */
const char *mbpt_last_error(const mbpt_context *ctx);
/* Replace the interaction (copied).  Affects task sets created afterwards and
 * the next integrate call of existing ones. */
int mbpt_set_interaction(mbpt_context *ctx, const mbpt_interaction *v);
/* Switch integrand precision (MBPT_FP64 / MBPT_FP32) for later calls. */
int mbpt_set_precision(mbpt_context *ctx, int precision);
/* Switch the single-particle spectrum (MBPT_SPECTRUM_FREE / _HF) for later
 * integrate calls of every task set of the context. */
int mbpt_set_spectrum(mbpt_context *ctx, int spectrum);
/* Regularised components (Sec. "Automated approach": the sensitivity to a
 * parameter added to every energy denominator): with n_eta in 1..4, every
 * later iteration also estimates, from the same samples, the integrals with
 * each energy denominator D_c replaced by D_c - k eta (k = 1..n_eta, eta > 0
 * in MeV; D_c < 0 wherever a Goldstone diagram is allowed, so the shift moves
 * every pole away).  The VEGAS grid adapts to the unregularised integrand; the
 * components are evaluated in fp64 whatever the precision, with the free
 * spectrum only (an HF context gives MBPT_ESTATE at integrate), and the server
 * refuses them.  n_eta = 0 switches them off.  A task set keeps the setting
 * its first iteration after a reset ran with: integrate returns MBPT_ESTATE
 * if it has changed since (call mbpt_reset).  EINVAL on n_eta outside 0..4 or
 * eta <= 0. */
int mbpt_set_regularization(mbpt_context *ctx, int n_eta, double eta);
/* FP32 precision: relative accuracy target per integrand value (0, the
 * default: only the near-Fermi-surface and small-denominator bands of the
 * context description).  With rel > 0 every fp32 sample also carries a
 * first-order bound of its relative error (from the regulator exponent, the
 * condition numbers of the energy and Yukawa denominators and the label sum's
 * cancellation, in units of the fp32 rounding unit) and is re-evaluated in
 * fp64 when the bound exceeds rel, so that each value is within rel of the
 * fp64 integrand.  Takes effect at the next integrate.  EINVAL if rel < 0. */
int mbpt_set_fp32_target(mbpt_context *ctx, double rel);

/* ---- diagram generator (host only, no context needed) --------------------- */
/* Number of two-body energy diagrams of an order (1, 1, 3, 39, 840 for orders
 * 1..5; Table I, N_diag). */
int mbpt_num_diagrams(int order, int *count);
/* The n x n line-count matrix of a diagram, row-major into M[order*order]:
 * M[u*order+v] lines run from time level u to level v (particle if u < v,
 * hole if u > v; order 1: one vertex with two hole self-lines, M = {2}).
 * Also returns the prefactor (1/2)^{n_eq} (-1)^{n_h + n_loop} if non-NULL. */
int mbpt_diagram_matrix(int order, int id, int *M, double *prefactor);
/* Label-sum statistics of a diagram: nonzero spin (NEUTRON) or spin-isospin
 * (NUCLEAR) label assignments, distinct isospin configurations consistent
 * with isospin conservation at every vertex, and compressed terms stored. */
int mbpt_diagram_label_stats(int order, int id, int matter, int *n_assign, int *n_isospin,
                             int *n_terms);
/* The label sum of a diagram as the polynomial it is in the vertex matrix
 * elements (eq:Dijkabc with the antisymmetrised vertex V_d - V_e): one row per
 * isospin configuration (one row in neutron matter), 2^order integer
 * coefficients c_E per row, where E runs over vertex subsets (bit v set:
 * vertex v contributes its exchange element V_e, else its direct element V_d)
 * and the configuration's sum is sum_E c_E prod_v (V_d,v or V_e,v).  coef is
 * caller-owned host memory of max_rows * 2^order doubles, row-major; rows are
 * ordered by the configuration's isospin mask over the kernel's line slots.
 * *n_rows receives the row count; MBPT_ENOMEM if it exceeds max_rows
 * (nothing written then).  coef may be NULL to query n_rows only. */
int mbpt_diagram_label_poly(int order, int id, int matter, double *coef, int max_rows,
                            int *n_rows);

/* Diagram groups of an order: the diagrams with p particle-carried loops
 * (the cycle rank of their particle-line subgraph), ascending ids into
 * caller-owned ids[cap]; *n receives the member count (0 for an empty group;
 * orders 1..5 have 1, 1, 2, 4, 5 non-empty groups, Table I's N_grp). */
int mbpt_group_members(int order, int p, int *ids, int cap, int *n);

/* ---- task sets ------------------------------------------------------------ */
/* A task set is the unit of batching: its tasks may mix orders, diagrams,
 * diagram groups, densities and proton fractions (one matter per set), and
 * mbpt_integrate runs all of them together, in BATCHED / GRAPH mode with one
 * sample launch per order present per iteration and one iteration-end launch
 * for all tasks.  It takes the place of a separate batch call over
 * (diagram set, n, x) triples: give each triple a task of one set.
 * Create a set of tasks (copied).  EINVAL on an unknown diagram, order outside
 * 1..5, density <= 0, proton fraction outside [0,1], or NEUTRON with x != 0. */
int mbpt_create_task_set(mbpt_context *ctx, const mbpt_task_desc *tasks, int n_tasks,
                         mbpt_task_set **out);
/* A diagram given by its lines and vertices (Sec. "Automated approach": a
 * diagram is read from its table of lines and vertices).  order: n = 1..5
 * vertices at time levels 0..n-1, bottom first.  nlines: must be 2n (<= 10).
 * Line l runs from level line_from[l] to level line_to[l]: a particle line if
 * from < to, a hole line if from > to (first order: two hole self-lines
 * 0 -> 0).  vertex[v] = {o1, o2, i1, i2}: the line ids of the antisymmetrised
 * matrix element <o1 o2|V(1 - P12)|i1 i2> at vertex v (o1, o2 leave v; i1, i2
 * enter v).  Dimensions 3(n + 1) <= 18.  Entries beyond nlines / order are
 * ignored. */
typedef struct mbpt_diagram_desc {
  int order;
  int nlines;
  int line_from[10];
  int line_to[10];
  int vertex[5][4];
} mbpt_diagram_desc;

/* Create a set of one task per descriptor (density 0.16 fm^-3, x = 0,
 * task_key = position; move them with mbpt_set_density / _asymmetry).  Each
 * descriptor is validated -- order 1..5, nlines = 2 order, levels in range,
 * no self-line above first order, two lines leaving and two entering every
 * vertex, vertex slots naming four distinct lines that leave (o1, o2) or
 * enter (i1, i2) it, all vertices connected -- else MBPT_EINVAL with the
 * reason in mbpt_last_error.  A two-body energy diagram is fixed by its
 * line-count matrix (relabelling lines, or exchanging a vertex's incoming
 * pair, which flips the sign of the matrix element and of the closed-loop
 * count together, leaves its value unchanged), so a valid descriptor runs the
 * library's compiled form of the generator diagram with the same matrix: its
 * label list (the nonzero spin(-isospin) assignments) is derived, not
 * supplied, and its samples are those of that generator id. */
int mbpt_create_diagram_set(mbpt_context *ctx, const mbpt_diagram_desc *descs, int n, int matter,
                            mbpt_task_set **out);
/* Validate one descriptor and return the generator id of its diagram (the
 * same checks; EINVAL without a message, as no context is involved). */
int mbpt_diagram_desc_id(const mbpt_diagram_desc *desc, int *id);
/* The generator's own descriptor of diagram `id` of an order (lines in the
 * compiled order: particles, then holes). */
int mbpt_diagram_desc_of(int order, int id, mbpt_diagram_desc *out);
/* Convenience: the listed generator diagrams of one order (ids NULL = all) at
 * density 0.16 fm^-3, x = 0, task_key = position in the list. */
int mbpt_create_diagram_set_from_order(mbpt_context *ctx, int order, const int *ids, int n_ids,
                                       int matter, mbpt_task_set **out);
void mbpt_task_set_destroy(mbpt_task_set *set);
int mbpt_task_count(const mbpt_task_set *set, int *n);
/* Move every task of the set to a new density [fm^-3] or proton fraction.
 * The VEGAS grids and the Philox iteration words are kept (warm start: the
 * next iteration starts from the adapted grid with fresh random numbers);
 * the running sums, counters and iteration logs restart, so later results
 * estimate the new EOS point from its own iterations only.  EINVAL on
 * density <= 0, x outside [0, 1], or x != 0 in a NEUTRON set. */
int mbpt_set_density(mbpt_task_set *set, double density);
int mbpt_set_asymmetry(mbpt_task_set *set, double proton_fraction);
int mbpt_set_launch_mode(mbpt_task_set *set, int mode);
/* Training and evaluation phases (Sec. "MC integration: PVegas"): with
 * train_iters > 0 the first train_iters iterations of every task after a
 * reset or an EOS-point move adapt its grid (training); from then on the grid
 * is frozen and the estimate, its sigma and chi2/dof combine the evaluation
 * iterations only (the training iterations stay in mbpt_iteration_log).
 * Until the first evaluation iteration the result combines the training
 * iterations.  0 (default): every iteration adapts the grid and is combined.
 * Applies from the set's next iteration.  EINVAL if train_iters < 0. */
int mbpt_set_training(mbpt_task_set *set, int train_iters);
/* Work decomposition: threads per block (64..256, multiple of 64; the sample
 * kernels are built for at most 256) and samples per thread per work item
 * (1..256).  EINVAL outside these ranges.  Without this call the block has
 * 256 threads and the samples per thread are chosen at mbpt_bind_workspace
 * for the launch mode the set has then: the larger of a task's samples over
 * about two blocks per CU (at most 16) and one launch's samples (one task in
 * the per-task mode, all tasks of an order otherwise) over about 16 blocks
 * per CU (at most 256).  A later mbpt_set_launch_mode keeps that choice.
 * ESTATE for smaller work items than the bound workspace was sized for. */
int mbpt_set_blocking(mbpt_task_set *set, int threads_per_block, int samples_per_thread);
/* The work decomposition in effect (the automatic choice once bound). */
int mbpt_get_blocking(const mbpt_task_set *set, int *threads_per_block, int *samples_per_thread);

/* Device workspace bytes needed for up to max_samples_per_iter samples per
 * task and iteration and up to max_iters stored per-iteration estimates. */
int mbpt_workspace_query(const mbpt_task_set *set, uint64_t max_samples_per_iter, int max_iters,
                         size_t *bytes);
/* Bind caller-owned device memory (256-byte aligned, >= the queried size for
 * the limits passed to the query).  Uploads descriptors and resets every grid
 * to uniform and every task to iteration 0.  ENOMEM if too small. */
int mbpt_bind_workspace(mbpt_task_set *set, void *device_ptr, size_t bytes,
                        uint64_t max_samples_per_iter, int max_iters);
/* Reset grids to uniform and iteration counters / sums to zero. */
int mbpt_reset(mbpt_task_set *set);

/* ---- integration ---------------------------------------------------------- */
/* Run `iters` VEGAS iterations of samples_per_iter samples for every task,
 * continuing from the current grids and iteration counters (so repeated calls
 * resume exactly).  Blocks until done.  per_task[n_tasks] receives the
 * cumulative result of each task (may be NULL); total (may be NULL) receives
 * the sum over tasks (sigmas in quadrature).  ESTATE without a workspace,
 * ENOMEM if samples_per_iter or the iteration count exceeds the bound limits,
 * ENUMERIC on a non-finite estimate. */
int mbpt_integrate(mbpt_task_set *set, uint64_t samples_per_iter, int iters,
                   mbpt_result *per_task, mbpt_result *total);
/* Per-iteration estimates of a task: I[k], var[k] for the iterations stored
 * so far (at most max_iters); *count receives how many were written. */
int mbpt_iteration_log(mbpt_task_set *set, int task, double *I, double *var, int cap,
                       int *count);
/* Integrand weights (Jacobian included) of samples [first, first+count) of
 * iteration `iter` of one task with its current grid, written to host memory.
 * For per-sample parity checks. */
int mbpt_dump_samples(mbpt_task_set *set, int task, uint32_t iter, uint64_t first,
                      uint64_t count, double *w_host);
/* HF self-energy Sigma_tau(k_i) [MeV] of a task at the spline nodes
 * k_i = i * (*h), i = 0..512 (eq:spe; tau 0 neutron, 1 proton, proton only in
 * NUCLEAR sets), written to sigma_host (513 doubles, caller-owned host
 * memory); computes the tables first if needed.  MBPT_ESTATE unless the
 * context's spectrum is HF and a workspace is bound.  Blocks on the stream. */
int mbpt_hf_nodes(mbpt_task_set *set, int task, int tau, double *sigma_host, double *h);
/* Regularised components of samples [first, first+count) of iteration `iter`
 * of one task (see mbpt_set_regularization; Jacobian included), into
 * caller-owned host memory wreg_host[count * n_eta], row-major
 * (wreg_host[i * n_eta + k]: component k + 1 of sample first + i).
 * MBPT_ESTATE without a workspace or without regularised components (or with
 * the HF spectrum).  Blocks on the stream. */
int mbpt_dump_samples_reg(mbpt_task_set *set, int task, uint32_t iter, uint64_t first,
                          uint64_t count, double *wreg_host);
/* Per-iteration estimates of the regularised components of a task for the
 * iterations stored since the last reset (at most max_iters, oldest first),
 * n_eta + 1 columns: I[i * (n_eta + 1) + k], var[i * (n_eta + 1) + k] for
 * component k + 1 (k < n_eta; shifted sums over the same samples as the main
 * estimate, with its shift), and in column n_eta the extrapolation to zero
 * shift, integrated per sample as sum_k a_k w_k (a_k: the weights with which
 * the equal-weight least-squares polynomial of degree min(2, n_eta - 1) in
 * eta_k = k eta through the components takes its value at eta = 0; for three
 * components 3, -3, 1), so that its variance carries the components'
 * correlation.  *count receives the iterations written (0 if none ran with
 * components).  I, var: host memory of cap * (n_eta + 1) doubles, may be
 * NULL. */
int mbpt_regularized_log(mbpt_task_set *set, int task, double *I, double *var, int cap,
                         int *count);
/* Cumulative regularised components of a task and their extrapolation to
 * eta = 0 (Sec. III.A: a quadratic fitted to the components).  Each
 * component, and the extrapolation (column n_eta of mbpt_regularized_log),
 * combines the logged iterations from index skip_iters on by inverse
 * variance, into E[n_eta] +- sigma[n_eta] and E0 +- sigma0 (each may be
 * NULL).  MBPT_ESTATE without logged components or with no positive variance
 * after skip_iters. */
int mbpt_regularized(mbpt_task_set *set, int task, int skip_iters, double *E, double *sigma,
                     double *E0, double *sigma0);
/* One-shot batch over many (diagram, EOS point) tasks: a task set of the n
 * tasks is created, bound to the caller's device workspace (bytes from
 * mbpt_batch_workspace_query for the same tasks, samples and iterations),
 * integrated from uniform grids for `iters` iterations of samples_per_iter
 * samples each with one sample launch per order per iteration (BATCHED), and
 * destroyed.  out[n] receives the per-task results (may be NULL), *total their
 * sum (may be NULL).  The workspace is borrowed for the call only.  The tasks
 * must share one matter (EINVAL otherwise); other errors as
 * mbpt_create_task_set, mbpt_bind_workspace and mbpt_integrate. */
int mbpt_batch_workspace_query(mbpt_context *ctx, const mbpt_task_desc *tasks, int n_tasks,
                               uint64_t samples_per_iter, int iters, size_t *bytes);
int mbpt_integrate_batch(mbpt_context *ctx, const mbpt_task_desc *tasks, int n_tasks,
                         uint64_t samples_per_iter, int iters, void *device_ptr, size_t bytes,
                         mbpt_result *out, mbpt_result *total);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): mbpt_integrate
 * on a set that has no workspace bound, with the set's device state held in a
 * static device array of MBPT_NOALLOC_SCRATCH_BYTES that the library keeps on
 * each GPU it runs on until the process ends.  Each call starts every task of
 * the set from a uniform grid at iteration 0, runs `iters` iterations on the
 * context stream and returns the results as mbpt_integrate does (same work
 * decomposition as a workspace bound with max_samples_per_iter =
 * samples_per_iter, so the same estimates up to the order of the fp64
 * histogram atomics); nothing persists in the set, which is left unbound
 * (mbpt_iteration_log, mbpt_get_grid and mbpt_dump_samples still need a
 * bound workspace).  No device memory, event or graph is created: launches
 * are neither graph-captured nor timed.  Every call on one GPU uses that GPU's
 * one array, which keeps the last call's contents (each call initialises what
 * it reads): calls that overlap on one GPU, from two host threads or on two
 * streams, race and corrupt each other's results.  EINVAL on a null set,
 * iters < 1 or samples_per_iter < 2; ESTATE if a workspace is bound; ENOMEM,
 * with the byte counts in mbpt_last_error, if the set needs more scratch at
 * this sample and iteration count than the array holds. */
#define MBPT_NOALLOC_SCRATCH_BYTES (32u << 20)
int mbpt_integrate_noalloc(mbpt_task_set *set, uint64_t samples_per_iter, int iters,
                           mbpt_result *per_task, mbpt_result *total);

/* Grid of a task (ndim x (n_bins+1) edges, host memory) for checkpointing,
 * and its restore.  ndim = 3 (order + 1). */
int mbpt_get_grid(mbpt_task_set *set, int task, double *edges_host);
int mbpt_set_grid(mbpt_task_set *set, int task, const double *edges_host);

/* Autotuner: times one iteration of the whole set for each candidate work
 * decomposition (threads per block in {64, 128, 256} x samples per thread in
 * {4, 8, 16, 32, 64, 128, 256}, limited to what the bound workspace holds), keeps the
 * fastest (mbpt_set_blocking) and resets the set (grids uniform, iteration 0),
 * so tuning never leaks into results.  The choice is cached per (matter,
 * precision, launch mode, orders present, samples_per_iter); a cached choice
 * is applied without timing.  Outputs (may be NULL): the chosen shape and its
 * sample-kernel milliseconds per iteration.  ESTATE without a workspace. */
int mbpt_autotune(mbpt_task_set *set, uint64_t samples_per_iter, int *threads_per_block,
                  int *samples_per_thread, double *ms_per_iter);

/* Timing of the sample kernels since the last call (HIP events on the
 * context stream): launches, total kernel milliseconds, samples evaluated,
 * and algorithmic FLOPs per evaluation counted from the descriptors (FMA = 2,
 * add/mul = 1, each exp/sqrt/sincos/division = 1). */
int mbpt_kernel_stats(mbpt_context *ctx, uint64_t *launches, double *kernel_ms,
                      uint64_t *evals, double *flops);
/* The algorithmic FLOP model behind those figures for one diagram (host only,
 * no context): *pre FLOPs every sample costs (VEGAS map, loop and line
 * momenta, Pauli tests, accumulation), *post those of a sample past the Pauli
 * test (denominators, matrix elements, monomial tables, weight), *per_unit
 * those of one label unit evaluated (an isospin configuration of the
 * polynomial form, label_mode 0, or one compressed assignment term, label_mode
 * 1), *units the diagram's label units (nuclear matter with the free spectrum
 * and label_mode 0 evaluates one polynomial per passing sample, the cycle form
 * of the label sum: 1 unit).  FMA = 2, add/mul = 1, each
 * exp/sqrt/sin/cos/division = 1.  mbpt_kernel_stats multiplies them with the
 * device's per-task counts of samples, passing samples and units evaluated.
 * EINVAL on an unknown diagram or a bad matter, label_mode, reg_exp (even,
 * 2..16) or spectrum. */
int mbpt_diagram_flops(int order, int id, int matter, int label_mode, int reg_exp, int spectrum,
                       double *pre, double *post, double *per_unit, double *units);
/* Algorithmic FLOPs and transcendental count per evaluation of a task. */
int mbpt_task_flops(const mbpt_task_set *set, int task, double *flops, double *transcendentals);

/* ---- serving: continuous batching of EOS-point requests ------------------ */
/* A server owns one device workspace (caller-owned, size from
 * mbpt_server_workspace_query) holding up to max_slots resident tasks.
 * Requests queue on submit; mbpt_server_step admits queued requests in
 * arrival order into free slots (by slot count, descriptor entries, table
 * arena bytes and work items), runs for every resident task the VEGAS
 * iterations its own estimates predict it still needs (the first three at
 * once, then ceil(k ((sigma/target)^2 - 1)), at most 32, within max_evals; one
 * launch per order present per iteration, one host synchronisation per step),
 * and retires tasks whose sigma reached max(sigma_rel |E|, sigma_abs) (after
 * at least three iterations) or whose evaluations reached max_evals.
 * A request's random stream is keyed by its ticket and its iteration plan by
 * its own state, so its result does not depend on what else is resident
 * (unless warm starts are on, see mbpt_server_set_warm_start).  The server
 * takes the free spectrum only (EINVAL / ESTATE with HF).
 *
 * Diagram groups (Sec. III.A; the grouping of mbpt_task_desc.group): a request
 * with group = 1 integrates the summed integrand of the order's diagrams with
 * diagram_id particle-carried loops in one VEGAS integral.  Its members take
 * consecutive entries of the server's descriptor table (24 entries per slot)
 * and their label tables bytes of the table arena (64 KiB per slot); a request
 * that would not fit an empty server is refused at submit (ENOMEM), others
 * wait for retirements.
 *
 * Regularised components (Sec. III.A): the context's mbpt_set_regularization
 * at mbpt_server_workspace_query and mbpt_server_create applies to every
 * request of the server for its lifetime (later changes of the context's
 * setting do not reach it).  Each request then also integrates the n_eta
 * shifted components and their extrapolation to zero shift over the same
 * samples (fp64 integrand, whatever the precision; see mbpt_regularized_log),
 * the host combines them by inverse variance every step, and the sigma target
 * applies to the extrapolation (see mbpt_server_poll_regularized) instead of
 * the main estimate. */
typedef struct mbpt_request {
  int order;
  int diagram_id;       /* diagram id, or with group = 1 particle-carried loops */
  int matter;
  double density;
  double proton_fraction;
  double sigma_rel;
  double sigma_abs;
  uint64_t samples_per_iter;
  uint64_t max_evals;
  int group;            /* 0: one diagram, 1: a diagram group */
} mbpt_request;

int mbpt_server_workspace_query(const mbpt_context *ctx, int max_slots,
                                uint64_t max_samples_per_iter, size_t *bytes);
int mbpt_server_create(mbpt_context *ctx, int max_slots, uint64_t max_samples_per_iter,
                       int max_queue, void *device_ptr, size_t bytes, mbpt_server **out);
void mbpt_server_destroy(mbpt_server *srv);
/* Queue a request; *ticket identifies it.  EBUSY if the queue is full. */
int mbpt_server_submit(mbpt_server *srv, const mbpt_request *req, uint64_t *ticket);
/* One scheduling step (admit, the planned iterations of all resident tasks,
 * retire).
 * *n_active receives the resident count after the round, *n_queued the queue
 * length. */
int mbpt_server_step(mbpt_server *srv, int *n_active, int *n_queued);
/* Warm start across EOS points (off by default): a newly admitted request
 * whose (order, diagram, matter) matches one retired earlier within
 * |n - n'| <= max_dn [fm^-3] and |x - x'| <= max_dx starts from the nearest
 * such request's adapted VEGAS grid instead of the uniform one (the hypercube
 * variables are scaled by the Fermi momenta, so neighbouring EOS points need
 * nearly the same grid).  The server keeps the grids of its last max_slots
 * retirements in its workspace.  With warm starts on, a result depends on
 * which requests retired before it was admitted.  max_dn <= 0 switches it
 * off.  *count of mbpt_server_warm_starts: admissions that started warm. */
int mbpt_server_set_warm_start(mbpt_server *srv, double max_dn, double max_dx);
int mbpt_server_warm_starts(const mbpt_server *srv, uint64_t *count);
/* Result of a ticket: *done = 1 once retired (result valid), else 0 (result
 * holds the running estimate if resident).  Times are host wall-clock seconds
 * from the server's creation: submit, admit and finish. */
int mbpt_server_poll(mbpt_server *srv, uint64_t ticket, mbpt_result *res, int *done,
                     double *t_submit, double *t_admit, double *t_finish);
/* Regularised components of a ticket (a server created with components):
 * E[n_eta] +- sigma[n_eta] per component and E0 +- sigma0 for the
 * extrapolation to zero shift (as in mbpt_regularized), each combined over
 * the request's iterations by inverse variance (iterations without variance
 * are exact).  Current values for a resident request, final ones once
 * retired; the pointers may be NULL.  EINVAL on an unknown ticket, ESTATE
 * without components or before the request's first iteration. */
int mbpt_server_poll_regularized(mbpt_server *srv, uint64_t ticket, double *E, double *sigma,
                                 double *E0, double *sigma0);

#ifdef __cplusplus
}
#endif
#endif /* MBPT_VEGAS_H */
