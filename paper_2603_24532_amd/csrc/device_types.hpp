// Device-side tables shared by the kernels and the host runtime that fills
// them.  Everything lives in the caller-bound workspace.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>
#include <type_traits>

namespace mbpt {

constexpr int kMaxBins = 128;
// Distinct label cycles of one diagram over all vertex-term choices (at most
// 33 at fifth order, 17 at fourth)
constexpr int kMaxCycles = 40;
constexpr int kBlockMax = 1024;

// Decoded loop coefficients per descriptor: 4 n sums (n <= 5) of at most
// 6 loops, padded to 8.
constexpr int kDescCoefSums = 20;
constexpr int kDescCoefStride = 8;

// Compiled diagram (read wave-uniformly through the scalar cache).
struct alignas(16) DiagDev {
  int order, nlines, nloops, ncuts;
  int group_off, ngroups, term_off, nterms;
  int loop_part[8];       // 1 if loop j is carried by a particle line
  uint32_t part_mask;     // bit l: line l is a particle line
  uint32_t line_mask;     // bits of all lines
  int id;                 // diagram id within its order (generator order)
  int pad1;
  double pref;            // (1/2)^{n_eq} (-1)^{n_h + n_loop} (2 pi)^{-3L}
  double pad0;
  // Signed 0/1/2 coefficients as loop bitmasks (bits 0-7: +1, 8-15: -1,
  // 16-23: +2, 24-31: -2):
  uint32_t lmask[10];     // line slot l momentum = sum_j c_lj k_j (slot j < L is loop j)
  uint32_t pmask_v[5];    // vertex v: 2p  = k_o1 - k_o2 = sum_j c_vj k_j
  uint32_t qmask_v[5];    // vertex v: 2p' = k_i1 - k_i2
  uint32_t cut_hole[4];   // D_c = sum_{holes in c} eps - sum_{particles in c} eps
  uint32_t cut_part[4];
  int pad3[2];
  // Label cycles (nuclear matter): choosing the direct or the exchange term
  // at every vertex (E, bit v = exchange at vertex v) ties the labels of the
  // lines into closed cycles.  cyc_mask[k]: the ncyc distinct cycles of all
  // E as line-slot masks; per E, the set of its cycles (bit k for cycle k)
  // and their number: cyc_e[E] = set | number << 56, and for diagrams with at
  // most 24 cycles also cyc_e32[E] = set | number << 24.
  int ncyc;
  int pad4;
  uint32_t cyc_mask[kMaxCycles];
  uint64_t cyc_e[32];
  uint32_t cyc_e32[32];
  // The loop coefficients of lmask / pmask_v / qmask_v decoded (the vertex
  // sums halved): sum s < 2 order is line slot s, then (2p, 2p') of each
  // vertex; fp64, then fp32.  The group kernels, whose member loop runs at
  // run time, read them through the scalar cache instead of decoding the
  // masks per sum and sample.
  double coef_d[kDescCoefSums][kDescCoefStride];
  float coef_f[kDescCoefSums][kDescCoefStride];
};

// Compile-time descriptor masks for the diagrams whose kernels are
// specialised: the one two-body diagram of orders 1 and 2, the three of
// order 3 and the 39 of order 4 (variant V = diagram id; V = -1 is the
// generic, descriptor-driven path).  From order 2 on they also hold the
// label-cycle words per vertex-term choice (cyc_e32, the packing of
// DiagDev::cyc_e32, plain loop order), and at orders 1-3 the coefficients
// of the neutron-matter label polynomial (label_coef_q2, its one isospin
// configuration).  The masks are those the generator
// compiles (loops first, plain loop order); with them the compiler folds the
// loop-momentum sums, drops the zero coefficients and shares equal vertex
// momenta.  Task-set and server creation check the generator's masks against
// these.
template <int ORDER, int V>
struct FixedMasks {
  static constexpr bool kFixed = false;
};
template <>
struct FixedMasks<1, 0> {
  static constexpr bool kFixed = true;
  static constexpr uint32_t line_mask = 0x3u, part_mask = 0x0u;
  static constexpr uint32_t lmask[2] = {0x1u, 0x2u};
  static constexpr uint32_t pmask_v[1] = {0x201u};
  static constexpr uint32_t qmask_v[1] = {0x201u};
  static constexpr uint32_t cut_hole[1] = {0x0u};
  static constexpr uint32_t cut_part[1] = {0x0u};
  static constexpr int loop_part[2] = {0, 0};
  static constexpr double label_coef_q2[2] = {4, -2};
};
template <>
struct FixedMasks<2, 0> {
  static constexpr bool kFixed = true;
  static constexpr uint32_t line_mask = 0xFu, part_mask = 0x9u;
  static constexpr uint32_t lmask[4] = {0x1u, 0x2u, 0x4u, 0x106u};
  static constexpr uint32_t pmask_v[2] = {0x1000006u, 0x402u};
  static constexpr uint32_t qmask_v[2] = {0x402u, 0x1000006u};
  static constexpr uint32_t cut_hole[1] = {0x6u};
  static constexpr uint32_t cut_part[1] = {0x9u};
  static constexpr int loop_part[3] = {1, 0, 0};
  static constexpr uint32_t cyc_e32[4] = {0x2000003u, 0x1000004u, 0x1000004u, 0x2000018u};
  static constexpr double label_coef_q2[4] = {4, -2, -2, 4};
};
template <>
struct FixedMasks<3, 0> {
  static constexpr bool kFixed = true;
  static constexpr uint32_t line_mask = 0x3Fu, part_mask = 0x11u;
  static constexpr uint32_t lmask[6] = {0x1u, 0x2u, 0x4u, 0x8u, 0x10Cu, 0x20Cu};
  static constexpr uint32_t pmask_v[3] = {0x100000Cu, 0x200000Cu, 0x804u};
  static constexpr uint32_t qmask_v[3] = {0x200000Cu, 0x804u, 0x100000Cu};
  static constexpr uint32_t cut_hole[2] = {0x22u, 0xCu};
  static constexpr uint32_t cut_part[2] = {0x11u, 0x11u};
  static constexpr int loop_part[4] = {1, 0, 0, 0};
  static constexpr uint32_t cyc_e32[8] = {0x2000003u, 0x1000004u, 0x1000004u, 0x2000018u,
                                          0x1000004u, 0x2000060u, 0x2000180u, 0x1000004u};
  static constexpr double label_coef_q2[8] = {4, -2, -2, 4, -2, 4, 4, -2};
};
template <>
struct FixedMasks<3, 1> {
  static constexpr bool kFixed = true;
  static constexpr uint32_t line_mask = 0x3Fu, part_mask = 0x31u;
  static constexpr uint32_t lmask[6] = {0x1u, 0x2u, 0x4u, 0x8u, 0x803u, 0x10Cu};
  static constexpr uint32_t pmask_v[3] = {0x8010402u, 0x201u, 0x804u};
  static constexpr uint32_t qmask_v[3] = {0x402u, 0x8000003u, 0x100000Cu};
  static constexpr uint32_t cut_hole[2] = {0x6u, 0xCu};
  static constexpr uint32_t cut_part[2] = {0x30u, 0x21u};
  static constexpr int loop_part[4] = {1, 0, 0, 0};
  static constexpr uint32_t cyc_e32[8] = {0x2000003u, 0x1000004u, 0x3000019u, 0x2000030u,
                                          0x1000004u, 0x20000C0u, 0x2000108u, 0x1000004u};
  static constexpr double label_coef_q2[8] = {4, -2, -8, 4, -2, 4, 4, -2};
};
template <>
struct FixedMasks<3, 2> {
  static constexpr bool kFixed = true;
  static constexpr uint32_t line_mask = 0x3Fu, part_mask = 0x33u;
  static constexpr uint32_t lmask[6] = {0x1u, 0x2u, 0x4u, 0x8u, 0x10Cu, 0x20Cu};
  static constexpr uint32_t pmask_v[3] = {0x100000Cu, 0x200000Cu, 0x804u};
  static constexpr uint32_t qmask_v[3] = {0x804u, 0x100000Cu, 0x200000Cu};
  static constexpr uint32_t cut_hole[2] = {0xCu, 0xCu};
  static constexpr uint32_t cut_part[2] = {0x11u, 0x22u};
  static constexpr int loop_part[4] = {1, 1, 0, 0};
  static constexpr uint32_t cyc_e32[8] = {0x2000003u, 0x1000004u, 0x1000004u, 0x2000018u,
                                          0x1000004u, 0x2000060u, 0x2000180u, 0x1000004u};
  static constexpr double label_coef_q2[8] = {4, -2, -2, 4, -2, 4, 4, -2};
};

}  // namespace mbpt

// the 39 fourth-order diagrams (generated; per-diagram fourth-order kernels)
#include "fixed_masks_o4.hpp"

namespace mbpt {

// FixedMasks that also hold the diagram's label cycles as compile-time
// constants (cyc_e32, the packing of DiagDev::cyc_e32): the generated
// fourth-order tables.
template <typename F, typename = void>
struct fixed_cycles : std::false_type {};
template <typename F>
struct fixed_cycles<F, std::void_t<decltype(F::cyc_e32)>> : std::true_type {};
// FixedMasks with the neutron-matter label coefficients (label_coef_q2).
template <typename F, typename = void>
struct fixed_labels : std::false_type {};
template <typename F>
struct fixed_labels<F, std::void_t<decltype(F::label_coef_q2)>> : std::true_type {};

}  // namespace mbpt

namespace mbpt {

// Isospin configuration: lines whose bit is set carry protons.  first/count:
// its explicit terms; coef_off: its 2^n factorised coefficients.
struct alignas(16) GroupDev {
  uint32_t tau;
  int first, count, coef_off;
};

// Factorised label-sum coefficients of one isospin configuration (2^n small
// integers) are stored as 2^n doubles followed by the same values as 2^n
// floats packed two per double slot, so either precision loads a contiguous
// run.
constexpr int coef_slots(int order) { return (1 << order) + ((1 << order) + 1) / 2; }

// Compressed label-sum term: multiplicity and 2-bit vertex codes
// (0: V_d, 1: -V_e, 2: V_d - V_e).
struct alignas(16) TermDev {
  double mult;
  uint32_t codes;
  float multf;  // mult as float for the fp32 integrand
};

// Interaction and medium constants common to a launch.
struct Phys {
  double V0;        // C0 * hbarc      [MeV fm^3]
  double Vy;        // Cy * hbarc      [MeV fm^3 * fm^-2]
  double m2;        // mpi^2
  double invLn;     // Lambda^{-reg_exp}
  double hb2m;      // hbar^2 / 2m
  int half_exp;     // reg_exp / 2
  int nb;           // bins per dimension
  uint32_t seed;
  int spectrum;     // 0 free, 1 Hartree-Fock (eq:spe)
};

// Hartree-Fock spectrum: cubic spline of Sigma_tau(k) on kHfIntervals equal
// steps of [0, kF,max + kHfRangeLambda * Lambda]; entry i holds the
// coefficients (a, b, c, d) of a + b t + c t^2 + d t^3 on [k_i, k_i + h],
// entry kHfIntervals holds (Sigma at the last node, 0, 0, 0).
constexpr int kHfIntervals = 512;
constexpr int kHfEntries = kHfIntervals + 1;
constexpr double kHfRangeLambda = 6.0;
constexpr int kHfGauss = 64;  // Gauss-Legendre points per dimension

// Diagram groups of orders 3 and 4 in nuclear matter hold one label-cycle
// table per member in LDS: at most this many members (the largest group has
// 22, checked when task sets and servers are created).
constexpr int kGroupCycleTables = 22;

// Regularised energy-denominator components (D_c -> D_c - k eta, k = 1..nreg).
constexpr int kMaxReg = 4;
// Sums per work item and per logged iteration of the regularised modes: a
// (sum, sum of squares) or (I, var) pair for each of the kMaxReg components,
// then one for the extrapolation to zero shift integrated per sample as
// sum_k reg_coef[k] w_k.
constexpr int kRegSums = 2 * (kMaxReg + 1);

// Iteration-end kernel: threads per task block and item loads in flight per
// thread.
constexpr int kFinishThreads = 1024;
constexpr int kFinishBatch = 4;

// One task: parameters (host-written) and running state (device-written).
struct alignas(16) TaskDev {
  int diag, nd, grid_off, hist_off;
  int item_begin, nitems, res_off, res_cap;  // work items [item_begin, +nitems)
  int store_begin;                           // partials/counters slot of the first item
  int hf_off;                                // first HF spline entry of this task
  uint32_t key;
  int order;
  uint64_t nsamples;
  double kF2[2];        // neutron, proton kF^2
  double Rh, Rp;        // loop radii for hole / particle loop lines
  double inv_density;
  double band_k, band_d;
  double rel_target;    // fp32: relative accuracy target per value (0: bands only)
  double hf_h, hf_inv_h;  // HF spline step and its inverse
  int ndiag;              // descriptors of the task from `diag` on (a diagram group: > 1)
  int train_iters;        // > 0: first train_iters iterations are training (see finish_iteration)
  int active;
  int plan;             // iterations of the current launch sequence it takes part in
  // state (written by the device)
  uint32_t iter;        // Philox iteration word of the next iteration
  int it_done;
  double shift;
  double wsum, wisum, wi2sum, zsum;
  int nzero;
  int ncomb;            // iterations combined into the running sums
  double lastI, lastV;
  uint64_t nevals, nfallback, npass, nterms;
};

// Work-item counters of the persistent launches, one per order (index 1..5),
// and the blocks per compute unit such a launch starts.
constexpr int kQueueSlots = 8;
constexpr int kPersistentBlocksPerCu = 16;

// Per work item counters: fp64 fallbacks, samples past the Pauli test, label
// terms evaluated.
constexpr int kItemCounters = 3;

struct KArgs {
  TaskDev *tasks;
  const DiagDev *diags;
  const GroupDev *groups;
  const TermDev *terms;
  double *grids;
  double *hists;
  double *partials;       // 4 doubles per work item
  uint64_t *counters;     // kItemCounters per work item
  double *reslog;         // (I, var) pairs
  const double *gcoef;    // factorised label-sum coefficients (see coef_slots)
  const int2 *olist;      // (first item, task), grouped by order, ascending items
  double *hf;             // HF spline entries, 4 doubles each
  double *cpart;          // per item: kRegSums component sums (regularised modes)
  double *creslog;        // per logged iteration: kRegSums, (I, var) pairs
  int *queue;             // per order: work-item counter of the persistent launches (may be null)
  double reg_eta;         // component k + 1 shifts every denominator by -(k + 1) reg_eta
  double reg_coef[kMaxReg];  // extrapolation weights (0 beyond nreg)
  int nreg;               // components (0: none)
  int pad_reg;
  int ntasks;
  int total_items;
  int spt;                // samples per thread per item
  int label_mode;         // 0 factorised label sums, 1 explicit terms
  Phys phys;
};

}  // namespace mbpt
