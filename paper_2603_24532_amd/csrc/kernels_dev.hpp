// Device code of the sample kernels for gfx950 (CDNA4): VEGAS Monte Carlo of
// MBPT energy diagrams.  Templates only (plus two small constant tables, one
// copy per code object); kernels_inst.hip instantiates them per order and
// matter, kernels.hip holds the iteration-end, HF and init kernels.
//
// One thread evaluates one sample at a time: Philox4x32-10 words -> VEGAS
// bins and fractions (grid in LDS) -> spherical loop momenta -> line momenta
// from the compiled descriptor -> Pauli factors (n_k for holes, 1 - n_k for
// particles) -> energy denominators (eq:Dijkabc, free spectrum) ->
// antisymmetrised matrix elements per vertex -> explicit spin(-isospin) label
// sum -> weight.  Sums of (w - c) and (w - c)^2 are kept per thread as plain
// sums (at most spt terms), merged across the wavefront, the block and the
// work items with compensated pair merges in a fixed order; refinement
// histograms of w^2 are privatised in LDS and merged with fp64 atomics.  The integrand is
// elementwise with no contraction, so it runs on the vector ALUs (no MFMA).
#pragma once
#include <hip/hip_runtime.h>

#include <type_traits>

#include "device_types.hpp"
#include "turn_table.hpp"
#include "kernels.hpp"

namespace mbpt {

// ---------------------------------------------------------------------------
// Philox4x32-10 (Salmon et al., SC'11)

__device__ __forceinline__ void philox4x32_10(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3,
                                              uint32_t k0, uint32_t k1, uint32_t *out) {
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    // 32 x 32 -> 64-bit products (one v_mad_u64_u32 each)
    const uint64_t p0 = static_cast<uint64_t>(0xD2511F53u) * c0;
    const uint64_t p1 = static_cast<uint64_t>(0xCD9E8D57u) * c2;
    // three-input XOR in one v_bitop3_b32 (truth table 0x96)
    const uint32_t n0 = __builtin_amdgcn_bitop3_b32(static_cast<uint32_t>(p1 >> 32), c1, k0, 0x96);
    const uint32_t n2 = __builtin_amdgcn_bitop3_b32(static_cast<uint32_t>(p0 >> 32), c3, k1, 0x96);
    c0 = n0;
    c1 = static_cast<uint32_t>(p1);
    c2 = n2;
    c3 = static_cast<uint32_t>(p0);
    k0 += 0x9E3779B9u;
    k1 += 0xBB67AE85u;
  }
  out[0] = c0;
  out[1] = c1;
  out[2] = c2;
  out[3] = c3;
}

// sin and cos of 2 pi k / MBPT_TURN_STEPS (copied into LDS by every sample
// kernel).
struct alignas(16) SinCos {
  double s, c;
};
constexpr int kTurnEntries = MBPT_TURN_STEPS + 1;
static __constant__ SinCos kTurnDev[kTurnEntries] = {MBPT_TURN_TABLE_INIT};
// 2^(j / 64), j = 0..63 (the table-driven exponential, copied into LDS beside
// the turn table)
constexpr int kExp2Entries = 64;
static __constant__ double kExp2Dev[kExp2Entries] = {MBPT_EXP2_TABLE_INIT};

__device__ __forceinline__ void load_turn_table(SinCos *dst, double *ex) {
  for (int i = threadIdx.x; i < kTurnEntries; i += blockDim.x) dst[i] = kTurnDev[i];
  for (int i = threadIdx.x; i < kExp2Entries; i += blockDim.x) ex[i] = kExp2Dev[i];
}

// What the integrand reads from LDS: the turn table, the 2^(j/64) table, the
// HF spline entries of the task (ntab isospin tables of kHfEntries x 4
// doubles, absent with the free spectrum) and the grid pairs (e_b + w_b 2^-33,
// w_b).  Block layout: turn table, 2^(j/64) table, HF tables, grid pairs, then
// the kernel's own scratch.
struct SampleLds {
  const SinCos *turn;
  const double *ex;
  const double *hf;
  const double2 *g;
  const void *cyc;  // label-cycle table(s) of the item's diagram(s) (cycle-form kernels)
};

// Diagram variant of a sample kernel's work items (template argument VF):
// a diagram id >= 0 fixes the descriptor masks at compile time (per-diagram
// kernels); kPerItem picks the variant per work item (with_variant).
constexpr int kPerItem = -2;

// The descriptor-driven single-diagram sample kernels of orders 4 and 5 read
// the loop coefficients of their momentum sums decoded in the descriptor
// (DiagDev::coef_d / coef_f) through the scalar cache, instead of decoding
// them from the bit masks per sum and sample on the scalar unit (so do the
// group kernels, per member).  Measured on MI355X against the masks: 9-13%
// faster at fourth order (per task, with components, neutron matter), 6-10%
// at fifth order, and 5-10% in the persistent kernels; against a table of
// the same values in LDS, 2-9% faster.
template <int ORDER, int P, int VF>
constexpr bool desc_coef() {
  return ORDER >= 4 && !(P == 3 || P == 4 || P == 6) && VF < 0;  // not the group modes
}

// Label-cycle bit vectors: bit k of CycWord<ORDER> stands for cycle k of a
// diagram (at most 17 at fourth order, 33 at fifth).
template <int ORDER>
using CycWord = std::conditional_t<(ORDER >= 5), uint64_t, uint32_t>;

// Fifth-order diagrams with at most 24 label cycles (696 of the 840) run the
// variant kNarrowCycles of the cycle-form kernels, with 32-bit cycle words
// (the packing of DiagDev::cyc_e32): half the scalar registers for the
// per-E words and single-word bit operations per term.
constexpr int kNarrowCycles = -4;
constexpr int kNarrowCycleMax = 24;
template <int ORDER, int V>
using CycWordV = std::conditional_t<(ORDER >= 5 && V != kNarrowCycles), uint64_t, uint32_t>;

// The nuclear-matter label sum runs in the cycle form (see label_sum) for
// single diagrams with the free spectrum and the factorised label sum.
template <int ORDER, int Q, bool G, bool X, bool HF>
constexpr bool cycle_form() {
  return Q == 4 && ORDER >= 2 && !G && !X && !HF;
}
// Diagram groups of orders 3 and 4 run the cycle form per member, with one
// cycle table per member in LDS (kGroupCycleTables of them).
template <int ORDER, int Q, bool X, bool HF>
constexpr bool group_cycle_form() {
  return Q == 4 && (ORDER == 3 || ORDER == 4) && !X && !HF;
}

// Bytes of the label-cycle table: one CycWord per set of lines.
template <int ORDER>
__host__ __device__ constexpr size_t cycle_table_bytes() {
  return (size_t{1} << (2 * ORDER)) * sizeof(CycWord<ORDER>);
}

// tab[s] = the cycles of diagram D that contain no line of the line set s
// (bit k set if (s & cycle k) = 0); built by the whole block.
template <typename W>
__device__ __forceinline__ void fill_cycle_table(const DiagDev *__restrict__ D, int nsets,
                                                 W *tab) {
  const int K = D->ncyc;
  for (int s = threadIdx.x; s < nsets; s += blockDim.x) {
    W w = 0;
    for (int k = 0; k < K; ++k)
      w |= (static_cast<uint32_t>(s) & D->cyc_mask[k]) == 0u ? (W(1) << k) : W(0);
    tab[s] = w;
  }
}
// In the words of the variant with_variant picks for D: 32 bits for a
// fifth-order diagram of at most kNarrowCycleMax cycles.
template <int ORDER>
__device__ __forceinline__ void build_cycle_table(const DiagDev *__restrict__ D, void *tab) {
  constexpr int NS = 1 << (2 * ORDER);
  if (ORDER >= 5 && D->ncyc <= kNarrowCycleMax)
    fill_cycle_table(D, NS, static_cast<uint32_t *>(tab));
  else
    fill_cycle_table(D, NS, static_cast<CycWord<ORDER> *>(tab));
}

// Bytes of the fixed tables at the start of a sample kernel's LDS.
__host__ __device__ constexpr size_t fixed_lds_bytes() {
  return kTurnEntries * sizeof(SinCos) + kExp2Entries * sizeof(double);
}

__host__ __device__ constexpr size_t hf_lds_doubles(int ntab) {
  return static_cast<size_t>(ntab) * kHfEntries * 4;
}

// Carves the block's dynamic LDS; returns the first free double after the
// grid pairs and fills the pointers.  Copies the turn and HF tables (the grid
// pairs are the caller's).
__device__ __forceinline__ double *carve_lds(const KArgs &a, const TaskDev *__restrict__ T,
                                             int ntab, int nd, double *smem, SampleLds &L,
                                             double2 *&g) {
  SinCos *turn = reinterpret_cast<SinCos *>(smem);
  double *ex = reinterpret_cast<double *>(turn + kTurnEntries);
  double *hf = ex + kExp2Entries;
  g = reinterpret_cast<double2 *>(hf + hf_lds_doubles(ntab));
  load_turn_table(turn, ex);
  if (ntab) {
    const double *src = a.hf + 4 * static_cast<size_t>(T->hf_off);
    const int n = static_cast<int>(hf_lds_doubles(ntab));
    for (int i = threadIdx.x; i < n; i += blockDim.x) hf[i] = src[i];
  }
  L.turn = turn;
  L.ex = ex;
  L.hf = ntab ? hf : nullptr;
  L.g = g;
  L.cyc = nullptr;
  return reinterpret_cast<double *>(g + nd * a.phys.nb);
}

// HF self-energy of table tau at |k| = kk from the LDS spline (constant
// beyond the last node).
__device__ __forceinline__ double hf_sigma(const double *__restrict__ hf, int tau, double kk,
                                           double inv_h) {
  const double u = kk * inv_h;
  int i = static_cast<int>(u);
  double t = u - static_cast<double>(i);
  if (i >= kHfIntervals) {
    i = kHfIntervals;
    t = 0.0;
  }
  const double *e = hf + 4 * (tau * kHfEntries + i);
  return fma(t, fma(t, fma(t, e[3], e[2]), e[1]), e[0]);
}

// sin(2 pi x) and cos(2 pi x) for x in [0, 1]: the nearest table angle
// 2 pi k / 128 rotated by the residual d, |d| <= pi / 128, whose sine and
// cosine - 1 come from their Taylor series (first omitted terms below 4e-19
// relative to sin d and 4e-18 absolute for cos d).
__device__ __forceinline__ void sincos_turn(const SinCos *__restrict__ tab, double x, double &s,
                                            double &c) {
  const double u = x * static_cast<double>(MBPT_TURN_STEPS);  // exact
  const double kf = rint(u);
  const double d = (u - kf) * (2.0 * M_PI / MBPT_TURN_STEPS);  // u - kf exact
  const double z = d * d;
  double ps = fma(z, -1.0 / 5040.0, 1.0 / 120.0);
  ps = fma(z, ps, -1.0 / 6.0);
  const double sd = fma(d * z, ps, d);
  double pc = fma(z, -1.0 / 720.0, 1.0 / 24.0);
  pc = fma(z, pc, -0.5);
  const double cm = z * pc;
  const int k = min(max(static_cast<int>(kf), 0), MBPT_TURN_STEPS);
  const SinCos t = tab[k];
  s = fma(t.s, cm, fma(t.c, sd, t.s));
  c = fma(t.c, cm, fma(-t.s, sd, t.c));
}

// Coefficient c in {0, +-1, +-2} of loop j in the uniform bitmask m (bits
// 0-7: +1, 8-15: -1, 16-23: +2, 24-31: -2) as a double, built from its bit
// pattern with scalar instructions only.  HALF: the coefficients halved
// (vertex relative momenta are half the difference of two line momenta).
template <bool HALF = false>
__device__ __forceinline__ double mask_coef(uint32_t m, int j) {
  uint32_t hi = 0u;
  hi = (m & (1u << j)) ? (HALF ? 0x3FE00000u : 0x3FF00000u) : hi;
  hi = (m & (1u << (8 + j))) ? (HALF ? 0xBFE00000u : 0xBFF00000u) : hi;
  hi = (m & (1u << (16 + j))) ? (HALF ? 0x3FF00000u : 0x40000000u) : hi;
  hi = (m & (1u << (24 + j))) ? (HALF ? 0xBFF00000u : 0xC0000000u) : hi;
  return __hiloint2double(static_cast<int>(hi), 0);
}

// sum_j c_j v_j over loops j < L (coefficients from the uniform bitmask m).
// SKIP0: m is a compile-time constant, so zero coefficients are left out
// (an fma with a zero coefficient is not foldable under IEEE rules).
template <int L, bool HALF = false, bool SKIP0 = false>
__device__ __forceinline__ void masked_sum(uint32_t m, const double (*k)[3], double *out) {
  double x = 0.0, y = 0.0, z = 0.0;
#pragma unroll
  for (int j = 0; j < L; ++j) {
    const double c = mask_coef<HALF>(m, j);
    if (SKIP0 && c == 0.0) continue;
    x = fma(c, k[j][0], x);
    y = fma(c, k[j][1], y);
    z = fma(c, k[j][2], z);
  }
  out[0] = x;
  out[1] = y;
  out[2] = z;
}

// sum_j c_j v_j over loops j < L with the coefficients c read from a table:
// the same operations, in the same order, as masked_sum of the mask they were
// decoded from (zero coefficients included).
template <int L>
__device__ __forceinline__ void table_sum(const double *c, const double (*k)[3], double *out) {
  double x = 0.0, y = 0.0, z = 0.0;
#pragma unroll
  for (int j = 0; j < L; ++j) {
    x = fma(c[j], k[j][0], x);
    y = fma(c[j], k[j][1], y);
    z = fma(c[j], k[j][2], z);
  }
  out[0] = x;
  out[1] = y;
  out[2] = z;
}
template <int L>
__device__ __forceinline__ void table_sum_f(const float *c, const float (*k)[3], float *out) {
  float x = 0.0f, y = 0.0f, z = 0.0f;
#pragma unroll
  for (int j = 0; j < L; ++j) {
    x = fmaf(c[j], k[j][0], x);
    y = fmaf(c[j], k[j][1], y);
    z = fmaf(c[j], k[j][2], z);
  }
  out[0] = x;
  out[1] = y;
  out[2] = z;
}

// Descriptor masks of diagram variant V: compile-time constants where
// FixedMasks<ORDER, V> has them, else read from the descriptor.
template <int ORDER, int V>
__device__ __forceinline__ uint32_t lmask_of(const DiagDev *__restrict__ D, int l) {
  if constexpr (FixedMasks<ORDER, V>::kFixed) return FixedMasks<ORDER, V>::lmask[l];
  else return D->lmask[l];
}
template <int ORDER, int V>
__device__ __forceinline__ uint32_t pmask_of(const DiagDev *__restrict__ D, int v) {
  if constexpr (FixedMasks<ORDER, V>::kFixed) return FixedMasks<ORDER, V>::pmask_v[v];
  else return D->pmask_v[v];
}
template <int ORDER, int V>
__device__ __forceinline__ uint32_t qmask_of(const DiagDev *__restrict__ D, int v) {
  if constexpr (FixedMasks<ORDER, V>::kFixed) return FixedMasks<ORDER, V>::qmask_v[v];
  else return D->qmask_v[v];
}
template <int ORDER, int V>
__device__ __forceinline__ uint32_t cut_hole_of(const DiagDev *__restrict__ D, int c) {
  if constexpr (FixedMasks<ORDER, V>::kFixed) return FixedMasks<ORDER, V>::cut_hole[c];
  else return D->cut_hole[c];
}
template <int ORDER, int V>
__device__ __forceinline__ uint32_t cut_part_of(const DiagDev *__restrict__ D, int c) {
  if constexpr (FixedMasks<ORDER, V>::kFixed) return FixedMasks<ORDER, V>::cut_part[c];
  else return D->cut_part[c];
}
template <int ORDER, int V>
__device__ __forceinline__ uint32_t line_mask_of(const DiagDev *__restrict__ D) {
  if constexpr (FixedMasks<ORDER, V>::kFixed) return FixedMasks<ORDER, V>::line_mask;
  else return D->line_mask;
}
template <int ORDER, int V>
__device__ __forceinline__ uint32_t part_mask_of(const DiagDev *__restrict__ D) {
  if constexpr (FixedMasks<ORDER, V>::kFixed) return FixedMasks<ORDER, V>::part_mask;
  else return D->part_mask;
}
template <int ORDER, int V>
__device__ __forceinline__ bool loop_part_of(const DiagDev *__restrict__ D, int j) {
  if constexpr (FixedMasks<ORDER, V>::kFixed) return FixedMasks<ORDER, V>::loop_part[j] != 0;
  else return D->loop_part[j] != 0;
}

// Runs f(std::integral_constant<int, V>) with the diagram variant of a task
// whose first descriptor is D: the one diagram of orders 1-2 (also as a
// single-member group), the diagram id at order 3 for single-diagram tasks,
// for the cycle form (CYF) at fifth order kNarrowCycles where the diagram
// has at most kNarrowCycleMax cycles, the generic path (-1) otherwise.  The
// branch is uniform per work item.
template <int ORDER, bool G, bool CYF = false, typename Fn>
__device__ __forceinline__ void with_variant(const DiagDev *__restrict__ D, Fn &&f) {
  if constexpr (ORDER <= 2) {
    f(std::integral_constant<int, 0>{});
  } else if constexpr (ORDER == 3 && !G) {
    // ids 0..2 are the order's only diagrams (the host validates task ids)
    if (D->id == 0) f(std::integral_constant<int, 0>{});
    else if (D->id == 1) f(std::integral_constant<int, 1>{});
    else f(std::integral_constant<int, 2>{});
  } else if constexpr (ORDER >= 5 && CYF) {
    if (D->ncyc <= kNarrowCycleMax) f(std::integral_constant<int, kNarrowCycles>{});
    else f(std::integral_constant<int, -1>{});
  } else {
    f(std::integral_constant<int, -1>{});
  }
}

// (p^2)^(reg_exp / 2) for the regulator exponent: HE > 0 is reg_exp / 2 fixed
// at compile time (the quartic regulator's kernels: no selects or loop, and
// vertices with equal momenta share their factors), HE = 0 takes it from the
// launch (a uniform loop).  Both multiply the same factors in the same order.
template <int HE, typename F>
__device__ __forceinline__ F reg_pow(F p2, int half_exp) {
  F r = p2;
  if constexpr (HE > 0) {
#pragma unroll
    for (int e = 1; e < HE; ++e) r *= p2;
  } else {
    for (int e = 1; e < half_exp; ++e) r *= p2;
  }
  return r;
}

// Square root of a finite a >= 0: hardware reciprocal square root refined by
// one coupled step on g = sqrt(a) and h = 1 / (2 sqrt(a)) (doubling its
// correct bits) and one Newton correction of g.  No rescaling: a is clamped to
// the smallest normal (so 0 gives 1.5e-154), and the squared momenta and
// (1 - c)(1 + c) that reach here are far from overflow.
__device__ __forceinline__ double sqrt_normal(double a) {
  a = fmax(a, 0x1p-1022);
  const double y = __builtin_amdgcn_rsq(a);
  double g = a * y;
  double h = 0.5 * y;
  const double r = fma(-g, h, 0.5);
  g = fma(g, r, g);
  h = fma(h, r, h);
  const double d = fma(-g, g, a);
  return fma(d, h, g);
}

// (s, c) += (s2, c2) with the rounding error of the leading parts kept
__device__ __forceinline__ void pair_merge(double &s, double &c, double s2, double c2) {
  const double t = s + s2;
  const double bp = t - s;
  const double err = (s - (t - bp)) + (s2 - bp);
  s = t;
  c = c + c2 + err;
}

// ---------------------------------------------------------------------------
// Per-sample integrand in fp64.  Returns the weight; writes the VEGAS bin of
// every dimension to bins[].

// Philox words -> VEGAS bins and mapped coordinates x (fp64, identical for
// both integrand precisions).  Returns the VEGAS Jacobian.
template <int ND>
__device__ __forceinline__ double vegas_map(const KArgs &a, const TaskDev *__restrict__ T,
                                            const double2 *__restrict__ g, uint64_t s,
                                            uint32_t iter, double *x, int *bins) {
  constexpr int NW = (ND + 3) / 4;
  const int nb = a.phys.nb;
  // counter (s lo, s hi, iteration, word block), key (seed, task)
  uint32_t wd[4 * NW];
#pragma unroll
  for (int j = 0; j < NW; ++j)
    philox4x32_10(static_cast<uint32_t>(s), static_cast<uint32_t>(s >> 32), iter,
                  static_cast<uint32_t>(j), a.phys.seed, T->key, wd + 4 * j);
  // bin b = floor(w nb / 2^32), fraction ((w nb mod 2^32) + 1/2) / 2^32.
  // y = w nb 2^-32 is exact in fp64 (at most 39 significant bits), so b (the
  // truncation of y >= 0) and y - b (v_fract_f64) come out exactly; the half
  // is folded into the grid pair's first entry, e_b + w_b 2^-33.  Returns
  // prod_m width_m; the factor nb^ND is in jac_const.
  double jac = 1.0;
  const double nbscale = static_cast<double>(nb) * 0x1p-32;
#pragma unroll
  for (int m = 0; m < ND; ++m) {
    const double y = static_cast<double>(wd[m]) * nbscale;
    const int b = static_cast<int>(y);
    const double r = __builtin_amdgcn_fract(y);
    const double2 ew = g[m * nb + b];
    x[m] = fma(r, ew.y, ew.x);
    jac *= ew.y;
    bins[m] = b;
  }
  return jac;
}

// Sample-independent part of the Jacobian of a task (uniform, hoisted out of
// the sample loops): nb^ND from the VEGAS map, 4 pi R_j^3 per loop from the
// spherical map (the rest, x0_j^2, is per sample), and 1/n.
template <int ORDER, int V>
__device__ __forceinline__ double jac_const(const KArgs &a, const TaskDev *__restrict__ T,
                                            const DiagDev *__restrict__ D) {
  constexpr int L = ORDER + 1;
  double c = T->inv_density;
  const double nb = static_cast<double>(a.phys.nb);
#pragma unroll
  for (int m = 0; m < 3 * L; ++m) c *= nb;
#pragma unroll
  for (int j = 0; j < L; ++j) {
    const double R = loop_part_of<ORDER, V>(D, j) ? T->Rp : T->Rh;
    c *= (4.0 * M_PI) * R * R * R;
  }
  return c;
}

// True if some label assignment survives the Pauli factors: neutron matter
// needs every line allowed as a neutron; nuclear matter needs one isospin
// configuration whose lines are all allowed.  A sample that fails does no
// further work (its weight is exactly zero); this also keeps structurally
// vanishing denominators (a one-particle-one-hole cut, where isospin
// conservation forces the same Fermi momentum on both lines) out of the
// division.
template <int Q>
__device__ __forceinline__ bool pauli_allowed(const KArgs &a, const DiagDev *__restrict__ D,
                                              uint32_t okN, uint32_t okP, uint32_t lmask) {
  if (Q == 2) return okN == lmask;
  const GroupDev *__restrict__ G = a.groups + D->group_off;
  bool any = false;
  for (int gi = 0; gi < D->ngroups; ++gi) {
    const uint32_t tau = G[gi].tau;
    any |= (((~tau & ~okN) | (tau & ~okP)) & lmask) == 0u;
  }
  return any;
}

// Spin(-isospin) label sum of one diagram, summed over the isospin
// configurations whose lines all pass the Pauli test.  Mode 0 evaluates each
// configuration's sum as the multilinear polynomial
//   sum_E c_E prod_{v not in E} V_d,v prod_{v in E} V_e,v
// (E: set of vertices taking the exchange term; c_E integer, compiled on the
// host from the nonzero label assignments): the monomials of the first
// ORDER/2 vertices and of the rest are tabulated once per sample, so a
// configuration costs 2^ORDER + 2^(ORDER - ORDER/2) multiply-adds however
// many assignments it holds.  Mode 1 walks the compressed assignment list.
template <typename F>
__device__ __forceinline__ F fma_t(F x, F y, F z) {
  return __builtin_fma(x, y, z);
}
template <>
__device__ __forceinline__ float fma_t<float>(float x, float y, float z) {
  return __builtin_fmaf(x, y, z);
}
// The 2^ORDER coefficients of a configuration in precision F (contiguous).
template <int ORDER, typename F>
__device__ __forceinline__ const F *coef_run(const double *block) {
  return block;
}
template <>
__device__ __forceinline__ const float *coef_run<1, float>(const double *block) {
  return reinterpret_cast<const float *>(block + 2);
}
template <>
__device__ __forceinline__ const float *coef_run<2, float>(const double *block) {
  return reinterpret_cast<const float *>(block + 4);
}
template <>
__device__ __forceinline__ const float *coef_run<3, float>(const double *block) {
  return reinterpret_cast<const float *>(block + 8);
}
template <>
__device__ __forceinline__ const float *coef_run<4, float>(const double *block) {
  return reinterpret_cast<const float *>(block + 16);
}
template <>
__device__ __forceinline__ const float *coef_run<5, float>(const double *block) {
  return reinterpret_cast<const float *>(block + 32);
}
template <typename F>
__device__ __forceinline__ F term_mult(const TermDev &t) {
  return t.mult;
}
template <>
__device__ __forceinline__ float term_mult<float>(const TermDev &t) {
  return t.multf;
}

// M[e] = prod_{v < NV} (bit v of e ? Ve[v] : Vd[v])
template <int NV, typename F>
__device__ __forceinline__ void monomials(const F *Vd, const F *Ve, F *M) {
  M[0] = F(1);
#pragma unroll
  for (int v = 0; v < NV; ++v) {
#pragma unroll
    for (int e = 0; e < (1 << v); ++e) {
      M[e + (1 << v)] = M[e] * Ve[v];
      M[e] = M[e] * Vd[v];
    }
  }
}

// Product of the energy denominators of one isospin configuration when the
// single-particle energies depend on isospin (HF spectrum in nuclear matter):
// D_c = Dn_c + sum over the cut's proton lines of +-(eps_p - eps_n), with
// Dn_c the denominator with every line a neutron.
template <int ORDER, int V>
__device__ __forceinline__ double group_den(const DiagDev *__restrict__ D, uint32_t tau,
                                            const double *Dn, const double *deps) {
  constexpr int NL = 2 * ORDER;
  double prod = 1.0;
#pragma unroll
  for (int c = 0; c < ORDER - 1; ++c) {
    const uint32_t hm = cut_hole_of<ORDER, V>(D, c) & tau, pm = cut_part_of<ORDER, V>(D, c) & tau;
    double Dc = Dn[c];
#pragma unroll
    for (int l = 0; l < NL; ++l) {
      uint32_t hi = (hm & (1u << l)) ? 0x3FF00000u : 0u;
      hi = (pm & (1u << l)) ? 0xBFF00000u : hi;
      Dc = fma(__hiloint2double(static_cast<int>(hi), 0), deps[l], Dc);
    }
    prod *= Dc;
  }
  return prod;
}

// True if some vertex-term choice E has every one of its label cycles
// allowed for at least one isospin (ab: cycles allowed as neutrons or as
// protons): exactly when some isospin configuration passes the Pauli test.
// Cycle set and cycle count of E (fourth order and below: at most 17
// cycles, the 32-bit packing).
// V: the diagram variant; where FixedMasks<ORDER, V> holds the cycles they
// are compile-time constants.
template <int ORDER, int V = -1>
__device__ __forceinline__ void cycles_of_e(const DiagDev *__restrict__ D, int E,
                                            CycWordV<ORDER, V> &m, uint32_t &n) {
  if constexpr (ORDER <= 4 && fixed_cycles<FixedMasks<ORDER, V>>::value) {
    const uint32_t w = FixedMasks<ORDER, V>::cyc_e32[E];
    m = w & 0xFFFFFFu;
    n = w >> 24;
  } else if constexpr (ORDER >= 5 && V == kNarrowCycles) {
    const uint32_t w = D->cyc_e32[E];
    m = w & 0xFFFFFFu;
    n = w >> 24;
  } else if constexpr (ORDER >= 5) {
    const uint64_t w = D->cyc_e[E];
    m = w & ((uint64_t{1} << 56) - 1);
    n = static_cast<uint32_t>(w >> 56);
  } else {
    const uint32_t w = D->cyc_e32[E];
    m = w & 0xFFFFFFu;
    n = w >> 24;
  }
}

template <int ORDER, int V = -1>
__device__ __forceinline__ bool cycle_any(const DiagDev *__restrict__ D, CycWordV<ORDER, V> ab) {
  bool any = false;
#pragma unroll
  for (int E = 0; E < (1 << ORDER); ++E) {
    CycWordV<ORDER, V> m;
    uint32_t n;
    cycles_of_e<ORDER, V>(D, E, m, n);
    any |= (ab & m) == m;
  }
  return any;
}

// 2^e for 0 <= e <= 30 from its bit pattern
template <typename F>
__device__ __forceinline__ F pow2_bits(uint32_t e) {
  return __hiloint2double(static_cast<int>((1023u + e) << 20), 0);
}
template <>
__device__ __forceinline__ float pow2_bits<float>(uint32_t e) {
  return __uint_as_float((127u + e) << 23);
}

template <int ORDER, typename W>
__device__ __forceinline__ uint32_t popc_w(W x) {
  if constexpr (sizeof(W) == 8) return static_cast<uint32_t>(__popcll(x));
  else return static_cast<uint32_t>(__popc(x));
}

// Cycle form of the nuclear-matter label sum.  Expanding every vertex into
// its direct and exchange terms, the choice E (bit v: exchange at vertex v)
// contributes (-1)^{|E|} prod_{v not in E} V_d,v prod_{v in E} V_e,v times
// the number of labellings that keep each of E's label cycles uniform with
// every line allowed: 2 spin states times the isospins (neutron, proton)
// allowed on all of the cycle's lines, per cycle.  With cA / cB the cycles
// whose lines are all allowed as neutrons / protons, E's count is 0 if a
// cycle is allowed for neither, else 2^{cycles(E) + cycles allowed for both}.
// The monomials carry the sign (-V_e) and are tabulated as in the
// configuration form; the counts are integers, so the sum equals the sum over
// isospin configurations up to rounding.
template <int ORDER, typename F, bool ABS = false, int V = -1>
__device__ __forceinline__ F label_sum_cycles(const DiagDev *__restrict__ D, const F *Vd,
                                              const F *Ve, CycWordV<ORDER, V> cA,
                                              CycWordV<ORDER, V> cB, F *absum = nullptr) {
  using W = CycWordV<ORDER, V>;
  constexpr int H = ORDER / 2;
  constexpr int NA = 1 << H, NB = 1 << (ORDER - H);
  F nVe[ORDER];
#pragma unroll
  for (int v = 0; v < ORDER; ++v) nVe[v] = -Ve[v];
  F MA[NA], MB[NB];
  monomials<H>(Vd, nVe, MA);
  monomials<ORDER - H>(Vd + H, nVe + H, MB);
  const W ab = cA | cB, both = cA & cB;
  F AA[ABS ? NA : 1], AB[ABS ? NB : 1];
  if constexpr (ABS) {
#pragma unroll
    for (int i = 0; i < NA; ++i) AA[i] = fabs(MA[i]);
#pragma unroll
    for (int i = 0; i < NB; ++i) AB[i] = fabs(MB[i]);
  }
  F acc = F(0), aacc = F(0);
#pragma unroll
  for (int eb = 0; eb < NB; ++eb) {
    F in = F(0), ain = F(0);
#pragma unroll
    for (int ea = 0; ea < NA; ++ea) {
      const int E = ea | (eb << H);
      W m;
      uint32_t n;
      cycles_of_e<ORDER, V>(D, E, m, n);
      const uint32_t e = popc_w<ORDER>(both & m) + n;
      const F c = (ab & m) == m ? pow2_bits<F>(e) : F(0);
      in = fma_t<F>(c, MA[ea], in);
      if constexpr (ABS) ain = fma_t<F>(c, AA[ea], ain);
    }
    acc = fma_t<F>(in, MB[eb], acc);
    if constexpr (ABS) aacc = fma_t<F>(ain, AB[eb], aacc);
  }
  if constexpr (ABS) *absum = aacc;
  return acc;
}

// ISO: divide each configuration's sum by its own denominators (Dn, deps).
// X: the explicit assignment list instead of the polynomial (compile-time, so
// a kernel holds the state of one form only).
// ABS: also the same sum with every term in absolute value (*absum), the
// scale against which the fp32 integrand's cancellation is judged.
template <int ORDER, int Q, typename F, bool ISO, bool X, int V, bool ABS = false>
__device__ __forceinline__ F label_sum(const KArgs &a, const DiagDev *__restrict__ D,
                                       const F *Vd, const F *Ve, uint32_t okN, uint32_t okP,
                                       uint32_t lmask, uint32_t &units, const double *Dn,
                                       const double *deps, F *absum = nullptr) {
  const GroupDev *__restrict__ G = a.groups + D->group_off;
  const int ngroups = D->ngroups;
  F acc = F(0), aacc = F(0);
  if constexpr (!X) {
    constexpr int H = ORDER / 2;
    constexpr int NA = 1 << H, NB = 1 << (ORDER - H);
    F MA[NA], MB[NB];
    monomials<H>(Vd, Ve, MA);
    monomials<ORDER - H>(Vd + H, Ve + H, MB);
    F AA[ABS ? NA : 1], AB[ABS ? NB : 1];
    if constexpr (ABS) {
#pragma unroll
      for (int i = 0; i < NA; ++i) AA[i] = fabs(MA[i]);
#pragma unroll
      for (int i = 0; i < NB; ++i) AB[i] = fabs(MB[i]);
    }
    // one isospin configuration's polynomial sum_E c_E prod V
    auto add_config = [&](const F *c, uint32_t tau) {
      F gs = F(0);
#pragma unroll
      for (int eb = 0; eb < NB; ++eb) {
        F in = F(0);
#pragma unroll
        for (int ea = 0; ea < NA; ++ea) in = fma_t<F>(c[eb * NA + ea], MA[ea], in);
        gs = fma_t<F>(in, MB[eb], gs);
      }
      if constexpr (ABS) {
#pragma unroll
        for (int eb = 0; eb < NB; ++eb) {
          F in = F(0);
#pragma unroll
          for (int ea = 0; ea < NA; ++ea) in = fma_t<F>(fabs(c[eb * NA + ea]), AA[ea], in);
          aacc = fma_t<F>(in, AB[eb], aacc);
        }
      }
      if constexpr (ISO) gs = static_cast<F>(static_cast<double>(gs) / group_den<ORDER, V>(D, tau, Dn, deps));
      acc += gs;
    };
    if constexpr (Q == 2 && fixed_labels<FixedMasks<ORDER, V>>::value) {
      // neutron matter, a diagram of the fixed tables: its one configuration
      // with compile-time coefficients
      F c[NA * NB];
#pragma unroll
      for (int i = 0; i < NA * NB; ++i)
        c[i] = static_cast<F>(FixedMasks<ORDER, V>::label_coef_q2[i]);
      ++units;
      add_config(c, 0u);
    } else {
      for (int gi = 0; gi < ngroups; ++gi) {
        const uint32_t tau = G[gi].tau;
        bool ok = true;
        if (Q == 4) ok = (((~tau & ~okN) | (tau & ~okP)) & lmask) == 0u;
        if (ok) {
          ++units;
          const F *__restrict__ C = coef_run<ORDER, F>(a.gcoef + G[gi].coef_off);
          F c[NA * NB];  // one batch of scalar loads, then the multiply-adds
#pragma unroll
          for (int i = 0; i < NA * NB; ++i) c[i] = C[i];
          add_config(c, tau);
        }
      }
    }
  } else {
    for (int gi = 0; gi < ngroups; ++gi) {
      const uint32_t tau = G[gi].tau;
      const int first = G[gi].first, cnt = G[gi].count;
      bool ok = true;
      if (Q == 4) ok = (((~tau & ~okN) | (tau & ~okP)) & lmask) == 0u;
      if (ok) {
        units += cnt;
        F gs = F(0);
        for (int t = first; t < first + cnt; ++t) {
          const TermDev tm = a.terms[t];
          F prod = F(1), aprod = F(1);
#pragma unroll
          for (int v = 0; v < ORDER; ++v) {
            const uint32_t code = (tm.codes >> (2 * v)) & 3u;
            const F ca = code != 1u ? F(1) : F(0);
            const F cb = code != 0u ? F(-1) : F(0);
            prod *= fma_t<F>(ca, Vd[v], cb * Ve[v]);
            if constexpr (ABS) aprod *= fma_t<F>(ca, fabs(Vd[v]), -cb * fabs(Ve[v]));
          }
          gs = fma_t<F>(term_mult<F>(tm), prod, gs);
          if constexpr (ABS) aacc = fma_t<F>(fabs(term_mult<F>(tm)), aprod, aacc);
        }
        if constexpr (ISO) gs = static_cast<F>(static_cast<double>(gs) / group_den<ORDER, V>(D, tau, Dn, deps));
        acc += gs;
      }
    }
  }
  if constexpr (ABS) *absum = aacc;
  return acc;
}

// exp(x) for x <= 0 by Tang's table-driven method (ACM TOMS 15, 1989): with
// k = rint(64 x / ln 2) = 64 m + j, exp(x) = 2^m 2^(j/64) e^r, r = x - k ln2/64
// (|r| <= ln2/128, reduced with the split constant so k HI is exact), e^r - 1
// from its degree-6 Taylor polynomial (truncation below 3e-20) and 2^(j/64)
// from the LDS table.  Within about one ulp; arguments below -1000 give 0.
__device__ __forceinline__ double exp_nonpos(double x, const double *ex) {
  x = fmax(x, -1000.0);
  const double kd = __builtin_rint(x * MBPT_INV_LN2_64);
  const int k = static_cast<int>(kd);
  const double r = fma(-kd, MBPT_LN2_64_LO, fma(-kd, MBPT_LN2_64_HI, x));
  double q = fma(r, 1.0 / 720.0, 1.0 / 120.0);
  q = fma(q, r, 1.0 / 24.0);
  q = fma(q, r, 1.0 / 6.0);
  q = fma(q, r, 0.5);
  q = fma(q, r, 1.0);
  const double t = ex[k & 63];
  return __builtin_ldexp(fma(t, r * q, t), k >> 6);
}

// 1/d from the hardware reciprocal and two Newton steps (d normal and finite;
// within about one ulp).
__device__ __forceinline__ double rcp_newton(double d) {
  double r = __builtin_amdgcn_rcp(d);
  double e = fma(-d, r, 1.0);
  r = fma(r, e, r);
  e = fma(-d, r, 1.0);
  return fma(r, e, r);
}

// Contribution of one diagram at the loop momenta k (prefactor, regulators,
// label sum and denominators; without the Jacobian and 1/n).  HF: single-
// particle energies of the Hartree-Fock spectrum (tables in LDS).
// REG: also add the regularised components w_k = w prod_c D_c / (D_c - k eta)
// to wr[k - 1].
template <int ORDER, int Q, bool HF, bool REG, bool X, bool PI, int V, int HE = 0, bool CY = false,
          bool SCR = false, bool TD = false>
__device__ __forceinline__ double diag_weight64(const KArgs &a, const TaskDev *__restrict__ T,
                                                const DiagDev *__restrict__ D,
                                                const SampleLds &Ls, const double (*k)[3],
                                                uint32_t &npass, uint32_t &nterms, double *wr) {
  constexpr int L = ORDER + 1;
  constexpr int NL = 2 * ORDER;
  constexpr int NC = ORDER - 1;

  // line momenta -> occupation tests and energies (HF: plus the self-energy
  // of a neutron, and for nuclear matter the proton-neutron difference)
  double eps[NL], deps[NL];
  uint32_t inN = 0, inP = 0;
#pragma unroll
  for (int l = 0; l < NL; ++l) {
    double kv[3];
    if (l < L) {
      // slot l < L carries loop momentum l itself
      kv[0] = k[l][0];
      kv[1] = k[l][1];
      kv[2] = k[l][2];
    } else {
      if constexpr (TD) table_sum<L>(D->coef_d[l], k, kv);
      else masked_sum<L, false, FixedMasks<ORDER, V>::kFixed>(lmask_of<ORDER, V>(D, l), k, kv);
    }
    const double k2 = kv[0] * kv[0] + kv[1] * kv[1] + kv[2] * kv[2];
    eps[l] = a.phys.hb2m * k2;
    deps[l] = 0.0;
    if constexpr (HF) {
      const double kk = sqrt_normal(k2);
      const double sn = hf_sigma(Ls.hf, 0, kk, T->hf_inv_h);
      if (Q == 4) deps[l] = hf_sigma(Ls.hf, 1, kk, T->hf_inv_h) - sn;
      eps[l] += sn;
    }
    inN |= (k2 < T->kF2[0]) ? (1u << l) : 0u;
    if (Q == 4) inP |= (k2 < T->kF2[1]) ? (1u << l) : 0u;
  }
  // a hole line is allowed if occupied, a particle line if empty
  const uint32_t lmask = line_mask_of<ORDER, V>(D), pmask = part_mask_of<ORDER, V>(D);
  const uint32_t okN = (inN ^ pmask) & lmask;
  const uint32_t okP = (inP ^ pmask) & lmask;
  CycWordV<ORDER, V> cA = 0, cB = 0;
  if constexpr (CY) {
    const CycWordV<ORDER, V> *tab = static_cast<const CycWordV<ORDER, V> *>(Ls.cyc);
    cA = tab[~okN & lmask];
    cB = tab[~okP & lmask];
    if (!cycle_any<ORDER, V>(D, cA | cB)) return 0.0;
  } else {
    if (!pauli_allowed<Q>(a, D, okN, okP, lmask)) return 0.0;
  }
  if constexpr (SCR) return 1.0;  // the Pauli screen (see screen_on)
  ++npass;

  // energy denominators (with every line a neutron when they depend on
  // isospin; the label sum then corrects them per configuration)
  constexpr bool iso_den = Q == 4 && HF;
  double dprod = 1.0;
  double Dn[NC > 0 ? NC : 1];
#pragma unroll
  for (int c = 0; c < NC; ++c) {
    const uint32_t hm = cut_hole_of<ORDER, V>(D, c), pm = cut_part_of<ORDER, V>(D, c);
    double Dc = 0.0;
#pragma unroll
    for (int l = 0; l < NL; ++l) {
      if constexpr (FixedMasks<ORDER, V>::kFixed) {
        if (hm & (1u << l)) Dc += eps[l];
        else if (pm & (1u << l)) Dc -= eps[l];
      } else {
        uint32_t hi = (hm & (1u << l)) ? 0x3FF00000u : 0u;
        hi = (pm & (1u << l)) ? 0xBFF00000u : hi;
        Dc = fma(__hiloint2double(static_cast<int>(hi), 0), eps[l], Dc);
      }
    }
    Dn[c] = Dc;
    dprod *= Dc;
  }

  // antisymmetrised matrix elements V_d = V(p, p'), V_e = V(p, -p') without
  // their regulators: the regulator product over all vertices factors out of
  // every label term and is applied once, exp(-sum_v (p^n + p'^n) / Lambda^n).
  // The 2n Yukawa denominators and the product of energy denominators are
  // inverted together with one division (prefix products), or (PI) with one
  // division per vertex pair (V_d, V_e) and one for the energy denominators,
  // which keeps 4n + 2 fewer doubles live.
  constexpr int NR = 2 * ORDER + 1;
  constexpr bool kPairInv = PI;
  double den[kPairInv ? 1 : NR];
  double Vd[ORDER], Ve[ORDER];
  double yreg = 0.0;
#pragma unroll
  for (int v = 0; v < ORDER; ++v) {
    double p[3], q[3];  // relative momenta p and p'
    if constexpr (TD) {
      table_sum<L>(D->coef_d[2 * ORDER + 2 * v], k, p);
      table_sum<L>(D->coef_d[2 * ORDER + 2 * v + 1], k, q);
    } else {
      masked_sum<L, true, FixedMasks<ORDER, V>::kFixed>(pmask_of<ORDER, V>(D, v), k, p);
      masked_sum<L, true, FixedMasks<ORDER, V>::kFixed>(qmask_of<ORDER, V>(D, v), k, q);
    }
    const double p2 = p[0] * p[0] + p[1] * p[1] + p[2] * p[2];
    const double q2 = q[0] * q[0] + q[1] * q[1] + q[2] * q[2];
    const double pq = p[0] * q[0] + p[1] * q[1] + p[2] * q[2];
    const double pn = reg_pow<HE>(p2, a.phys.half_exp), qn = reg_pow<HE>(q2, a.phys.half_exp);
    yreg = v == 0 ? pn + qn : yreg + (pn + qn);
    const double s2 = p2 + q2 + a.phys.m2;
    const double dd = s2 - 2.0 * pq, de = s2 + 2.0 * pq;
    if constexpr (kPairInv) {
      const double r = rcp_newton(dd * de);
      Vd[v] = a.phys.V0 + a.phys.Vy * (de * r);
      Ve[v] = a.phys.V0 + a.phys.Vy * (dd * r);
    } else {
      den[2 * v] = dd;
      den[2 * v + 1] = de;
    }
  }
  double rden;  // 1 / prod_c D_c (1 when the label sum divides per configuration)
  if constexpr (kPairInv) {
    rden = iso_den ? 1.0 : rcp_newton(dprod);
  } else {
    den[NR - 1] = iso_den ? 1.0 : dprod;
    double pre[NR];
    pre[0] = den[0];
#pragma unroll
    for (int i = 1; i < NR; ++i) pre[i] = pre[i - 1] * den[i];
    double inv = rcp_newton(pre[NR - 1]);
    double rinv[NR];
#pragma unroll
    for (int i = NR - 1; i > 0; --i) {
      rinv[i] = inv * pre[i - 1];
      inv *= den[i];
    }
    rinv[0] = inv;
#pragma unroll
    for (int v = 0; v < ORDER; ++v) {
      Vd[v] = a.phys.V0 + a.phys.Vy * rinv[2 * v];
      Ve[v] = a.phys.V0 + a.phys.Vy * rinv[2 * v + 1];
    }
    rden = rinv[NR - 1];
  }
  const double regall = exp_nonpos(-yreg * a.phys.invLn, Ls.ex);

  double acc;
  if constexpr (CY) {
    ++nterms;
    acc = label_sum_cycles<ORDER, double, false, V>(D, Vd, Ve, cA, cB);
  } else {
    acc = label_sum<ORDER, Q, double, iso_den, X, V>(a, D, Vd, Ve, okN, okP, lmask, nterms, Dn,
                                                     deps);
  }
  const double base = D->pref * regall * acc;
  if constexpr (REG) {
    for (int r = 0; r < a.nreg; ++r) {
      const double eta = (r + 1) * a.reg_eta;
      double pk = 1.0;
#pragma unroll
      for (int c = 0; c < NC; ++c) pk *= Dn[c] - eta;
      wr[r] += base / pk;
    }
  }
  return base * rden;
}

// One sample of a task: VEGAS map, loop momenta (radii from the first
// descriptor: the members of a diagram group share them), then the diagram,
// or (G) the task's T->ndiag group members summed.
// REG: the regularised components go to wr[0..nreg) (Jacobian and 1/n
// included).
template <int ORDER, int Q, bool HF, bool G, bool X, bool PI, int V, bool REG = false, int HE = 0,
          bool SCR = false, bool TD = false>
__device__ __forceinline__ double eval_fp64(const KArgs &a, const TaskDev *__restrict__ T,
                                            const DiagDev *__restrict__ D,
                                            const SampleLds &Ls, double jc, uint64_t s,
                                            uint32_t iter, int *bins, uint32_t &npass,
                                            uint32_t &nterms, double *wr = nullptr) {
  constexpr int L = ORDER + 1;
  constexpr int ND = 3 * L;
  double x[ND];
  double jac = vegas_map<ND>(a, T, Ls.g, s, iter, x, bins);

  // loop momenta: radius R x0, cos theta = 2 x1 - 1, azimuth 2 pi x2
  // (Jacobian 4 pi R^3 x0^2 per loop)
  double k[L][3];
  double x0p = 1.0;  // prod_j x0_j
#pragma unroll
  for (int j = 0; j < L; ++j) {
    const double R = loop_part_of<ORDER, V>(D, j) ? T->Rp : T->Rh;
    const double rad = R * x[3 * j];
    const double ct = 2.0 * x[3 * j + 1] - 1.0;
    const double st = sqrt_normal((1.0 - ct) * (1.0 + ct));
    double sp, cp;
    sincos_turn(Ls.turn, x[3 * j + 2], sp, cp);
    k[j][0] = rad * st * cp;
    k[j][1] = rad * st * sp;
    k[j][2] = rad * ct;
    x0p *= x[3 * j];
  }
  if constexpr (REG)
    for (int r = 0; r < kMaxReg; ++r) wr[r] = 0.0;
  double sum;
  if constexpr (G) {
    sum = 0.0;
    const int nd = T->ndiag;
    for (int di = 0; di < nd; ++di) {
      // the members' loop coefficients from their descriptors
      constexpr bool TDG = !FixedMasks<ORDER, V>::kFixed;
      if constexpr (group_cycle_form<ORDER, Q, X, HF>()) {
        SampleLds Lm = Ls;  // the member's cycle table
        Lm.cyc = static_cast<const char *>(Ls.cyc) + di * cycle_table_bytes<ORDER>();
        sum += diag_weight64<ORDER, Q, HF, REG, X, PI, V, HE, true, false, TDG>(
            a, T, D + di, Lm, k, npass, nterms, wr);
      } else {
        sum += diag_weight64<ORDER, Q, HF, REG, X, PI, V, HE, false, false, TDG>(
            a, T, D + di, Ls, k, npass, nterms, wr);
      }
    }
  } else {
    constexpr bool CY = cycle_form<ORDER, Q, false, X, HF>();
    sum = diag_weight64<ORDER, Q, HF, REG, X, PI, V, HE, CY, SCR, TD>(a, T, D, Ls, k, npass,
                                                                    nterms, wr);
    if constexpr (SCR) return sum;
  }
  const double scale = jac * (x0p * x0p) * jc;
  if constexpr (REG)
    for (int r = 0; r < kMaxReg; ++r) wr[r] *= scale;
  return scale * sum;
}

// fp32 counterpart of masked_sum
template <bool HALF = false>
__device__ __forceinline__ float mask_coef_f(uint32_t m, int j) {
  uint32_t bits = 0u;
  bits = (m & (1u << j)) ? (HALF ? 0x3F000000u : 0x3F800000u) : bits;
  bits = (m & (1u << (8 + j))) ? (HALF ? 0xBF000000u : 0xBF800000u) : bits;
  bits = (m & (1u << (16 + j))) ? (HALF ? 0x3F800000u : 0x40000000u) : bits;
  bits = (m & (1u << (24 + j))) ? (HALF ? 0xBF800000u : 0xC0000000u) : bits;
  return __uint_as_float(bits);
}

template <int L, bool HALF = false, bool SKIP0 = false>
__device__ __forceinline__ void masked_sum_f(uint32_t m, const float (*k)[3], float *out) {
  float x = 0.0f, y = 0.0f, z = 0.0f;
#pragma unroll
  for (int j = 0; j < L; ++j) {
    const float c = mask_coef_f<HALF>(m, j);
    if (SKIP0 && c == 0.0f) continue;
    x = fmaf(c, k[j][0], x);
    y = fmaf(c, k[j][1], y);
    z = fmaf(c, k[j][2], z);
  }
  out[0] = x;
  out[1] = y;
  out[2] = z;
}

// Per-sample integrand with fp32 arithmetic after the (fp64) VEGAS map; the
// Jacobian and the final weight stay fp64.  Sets `fallback` instead of
// returning a value when the sample lies in the band where fp32 cannot
// resolve the result to the target accuracy: a line within band_k kF^2 of a
// Fermi surface (the Pauli factor could flip), an energy denominator below
// band_d times the sum of its energies (cancellation), or a regulator exponent
// or reciprocal product outside the fp32 range.  The caller then evaluates the
// sample in fp64 from the same random words.
// fp32 contribution of one diagram at the loop momenta k (see
// diag_weight64); sets `fallback` instead when the sample needs fp64.
template <int ORDER, int Q, bool X, int V, int HE = 0, bool CY = false, bool SCR = false,
          bool TD = false>
__device__ __forceinline__ double diag_weight32(const KArgs &a, const TaskDev *__restrict__ T,
                                                const DiagDev *__restrict__ D,
                                                const SampleLds &Ls, const float (*k)[3],
                                                uint32_t &npass, uint32_t &nterms,
                                                bool &fallback) {
  constexpr int L = ORDER + 1;
  constexpr int NL = 2 * ORDER;
  constexpr int NC = ORDER - 1;
  const float kFn2 = static_cast<float>(T->kF2[0]), kFp2 = static_cast<float>(T->kF2[1]);
  const float bandk = static_cast<float>(T->band_k), bandd = static_cast<float>(T->band_d);
  const float hb2m = static_cast<float>(a.phys.hb2m);
  float eps[NL];
  uint32_t inN = 0, inP = 0;
  bool near = false;
#pragma unroll
  for (int l = 0; l < NL; ++l) {
    float kv[3];
    if (l < L) {
      kv[0] = k[l][0];
      kv[1] = k[l][1];
      kv[2] = k[l][2];
    } else {
      if constexpr (TD) table_sum_f<L>(D->coef_f[l], k, kv);
      else masked_sum_f<L, false, FixedMasks<ORDER, V>::kFixed>(lmask_of<ORDER, V>(D, l), k, kv);
    }
    const float k2 = kv[0] * kv[0] + kv[1] * kv[1] + kv[2] * kv[2];
    eps[l] = hb2m * k2;
    near |= fabsf(k2 - kFn2) < bandk * kFn2;
    inN |= (k2 < kFn2) ? (1u << l) : 0u;
    if (Q == 4) {
      near |= fabsf(k2 - kFp2) < bandk * kFp2;
      inP |= (k2 < kFp2) ? (1u << l) : 0u;
    }
  }
  if (near) {
    if constexpr (SCR) return 1.0;  // the Pauli screen (see screen_on)
    fallback = true;
    return 0.0;
  }
  const uint32_t lmask = line_mask_of<ORDER, V>(D), pmask = part_mask_of<ORDER, V>(D);
  const uint32_t okN = (inN ^ pmask) & lmask;
  const uint32_t okP = (inP ^ pmask) & lmask;
  CycWordV<ORDER, V> cA = 0, cB = 0;
  if constexpr (CY) {
    const CycWordV<ORDER, V> *tab = static_cast<const CycWordV<ORDER, V> *>(Ls.cyc);
    cA = tab[~okN & lmask];
    cB = tab[~okP & lmask];
    if (!cycle_any<ORDER, V>(D, cA | cB)) return 0.0;
  } else {
    if (!pauli_allowed<Q>(a, D, okN, okP, lmask)) return 0.0;
  }
  if constexpr (SCR) return 1.0;

  float dprod = 1.0f;
  float kcut = 0.0f;  // sum of the cuts' condition numbers (sum |eps|) / |D|
#pragma unroll
  for (int c = 0; c < NC; ++c) {
    const uint32_t hm = cut_hole_of<ORDER, V>(D, c), pm = cut_part_of<ORDER, V>(D, c);
    float Dc = 0.0f, Dabs = 0.0f;
#pragma unroll
    for (int l = 0; l < NL; ++l) {
      uint32_t bits = (hm & (1u << l)) ? 0x3F800000u : 0u;
      bits = (pm & (1u << l)) ? 0xBF800000u : bits;
      const float cf = __uint_as_float(bits);
      Dc = fmaf(cf, eps[l], Dc);
      Dabs = fmaf(fabsf(cf), eps[l], Dabs);
    }
    near |= fabsf(Dc) < bandd * Dabs;
    kcut = fmaf(Dabs, __builtin_amdgcn_rcpf(fabsf(Dc)), kcut);
    dprod *= Dc;
  }

  constexpr int NR = 2 * ORDER + 1;
  float den[NR];
  float yreg = 0.0f;  // sum of the regulator exponents
  float yscale[ORDER];  // |p|^2 + |p'|^2 + 2 |p.p'| + m^2: scale of the Yukawa denominators
  const float m2 = static_cast<float>(a.phys.m2);
#pragma unroll
  for (int v = 0; v < ORDER; ++v) {
    float p[3], q[3];
    if constexpr (TD) {
      table_sum_f<L>(D->coef_f[2 * ORDER + 2 * v], k, p);
      table_sum_f<L>(D->coef_f[2 * ORDER + 2 * v + 1], k, q);
    } else {
      masked_sum_f<L, true, FixedMasks<ORDER, V>::kFixed>(pmask_of<ORDER, V>(D, v), k, p);
      masked_sum_f<L, true, FixedMasks<ORDER, V>::kFixed>(qmask_of<ORDER, V>(D, v), k, q);
    }
    const float p2 = p[0] * p[0] + p[1] * p[1] + p[2] * p[2];
    const float q2 = q[0] * q[0] + q[1] * q[1] + q[2] * q[2];
    const float pq = p[0] * q[0] + p[1] * q[1] + p[2] * q[2];
    const float pn = reg_pow<HE>(p2, a.phys.half_exp), qn = reg_pow<HE>(q2, a.phys.half_exp);
    yreg = v == 0 ? pn + qn : yreg + (pn + qn);
    const float s2 = p2 + q2 + m2;
    den[2 * v] = s2 - 2.0f * pq;
    den[2 * v + 1] = s2 + 2.0f * pq;
    yscale[v] = s2 + 2.0f * fabsf(pq);
  }
  den[NR - 1] = dprod;
  float pre[NR];
  pre[0] = den[0];
#pragma unroll
  for (int i = 1; i < NR; ++i) pre[i] = pre[i - 1] * den[i];
  const float yexp = yreg * static_cast<float>(a.phys.invLn);
  near |= !(fabsf(pre[NR - 1]) > 1e-30f && fabsf(pre[NR - 1]) < 1e30f) || yexp > 80.0f;
  if (near) {
    fallback = true;
    return 0.0;
  }
  float inv = __builtin_amdgcn_rcpf(pre[NR - 1]);
  inv = inv * (2.0f - pre[NR - 1] * inv);  // one Newton step
  float rinv[NR];
#pragma unroll
  for (int i = NR - 1; i > 0; --i) {
    rinv[i] = inv * pre[i - 1];
    inv *= den[i];
  }
  rinv[0] = inv;
  const float V0 = static_cast<float>(a.phys.V0), Vy = static_cast<float>(a.phys.Vy);
  float Vd[ORDER], Ve[ORDER];
#pragma unroll
  for (int v = 0; v < ORDER; ++v) {
    Vd[v] = fmaf(Vy, rinv[2 * v], V0);
    Ve[v] = fmaf(Vy, rinv[2 * v + 1], V0);
  }
  const float regall = __expf(-yexp);

  float acc;
  const uint32_t nterms0 = nterms;
  if (T->rel_target > 0.0) {
    // relative-accuracy target per value: a first-order bound on the fp32
    // evaluation's relative error, in units of the fp32 rounding unit u:
    // the regulator exponent (its momenta carry a few u each), the cuts'
    // and the Yukawa denominators' condition numbers, the label sum's
    // cancellation (sum of |terms| / |sum|) and a constant for the rest
    float aabs;
    if constexpr (CY) {
      ++nterms;
      acc = label_sum_cycles<ORDER, float, true, V>(D, Vd, Ve, cA, cB, &aabs);
    } else {
      acc = label_sum<ORDER, Q, float, false, X, V, true>(a, D, Vd, Ve, okN, okP, lmask, nterms,
                                                          nullptr, nullptr, &aabs);
    }
    float ky = 0.0f;
#pragma unroll
    for (int v = 0; v < ORDER; ++v)
      ky = fmaf(yscale[v], rinv[2 * v] + rinv[2 * v + 1], ky);
    const float cancel = aabs * __builtin_amdgcn_rcpf(fabsf(acc));
    const float bound =
        0x1p-24f * (8.0f * yexp + 4.0f * kcut + 4.0f * ky + 8.0f * cancel + 64.0f);
    if (!(bound <= static_cast<float>(T->rel_target))) {
      nterms = nterms0;
      fallback = true;
      return 0.0;
    }
  } else {
    if constexpr (CY) {
      ++nterms;
      acc = label_sum_cycles<ORDER, float, false, V>(D, Vd, Ve, cA, cB);
    } else {
      acc = label_sum<ORDER, Q, float, false, X, V>(a, D, Vd, Ve, okN, okP, lmask, nterms,
                                                   nullptr, nullptr);
    }
  }
  ++npass;
  return D->pref * static_cast<double>(regall) * static_cast<double>(acc) *
         static_cast<double>(rinv[NR - 1]);
}

template <int ORDER, int Q, bool G, bool X, int V, int HE = 0, bool SCR = false, bool TD = false>
__device__ __forceinline__ double eval_fp32(const KArgs &a, const TaskDev *__restrict__ T,
                                            const DiagDev *__restrict__ D,
                                            const SampleLds &Ls, double jc, uint64_t s,
                                            uint32_t iter, int *bins, uint32_t &npass,
                                            uint32_t &nterms, bool &fallback) {
  constexpr int L = ORDER + 1;
  constexpr int ND = 3 * L;
  double x[ND];
  double jac = vegas_map<ND>(a, T, Ls.g, s, iter, x, bins);

  // loop momenta; the azimuth goes to the hardware sine/cosine in revolutions
  float k[L][3];
  double x0p = 1.0;  // prod_j x0_j
#pragma unroll
  for (int j = 0; j < L; ++j) {
    const double R = loop_part_of<ORDER, V>(D, j) ? T->Rp : T->Rh;
    const double rad64 = R * x[3 * j];
    x0p *= x[3 * j];
    const float rad = static_cast<float>(rad64);
    const float ct = static_cast<float>(2.0 * x[3 * j + 1] - 1.0);
    const float st = __builtin_sqrtf(fmaxf(0.0f, (1.0f - ct) * (1.0f + ct)));
    const float rev = static_cast<float>(x[3 * j + 2]);
    const float sp = __builtin_amdgcn_sinf(rev), cp = __builtin_amdgcn_cosf(rev);
    const float rs = rad * st;
    k[j][0] = rs * cp;
    k[j][1] = rs * sp;
    k[j][2] = rad * ct;
  }
  double sum;
  if constexpr (G) {
    sum = 0.0;
    const int nd = T->ndiag;
    // members' counts are kept aside until every member has passed: a sample
    // that falls back is counted once, by its fp64 re-evaluation
    uint32_t gpass = 0, gterms = 0;
    for (int di = 0; di < nd; ++di) {
      constexpr bool TDG = !FixedMasks<ORDER, V>::kFixed;
      if constexpr (group_cycle_form<ORDER, Q, X, false>()) {
        SampleLds Lm = Ls;  // the member's cycle table
        Lm.cyc = static_cast<const char *>(Ls.cyc) + di * cycle_table_bytes<ORDER>();
        sum += diag_weight32<ORDER, Q, X, V, HE, true, false, TDG>(a, T, D + di, Lm, k, gpass,
                                                                    gterms, fallback);
      } else {
        sum += diag_weight32<ORDER, Q, X, V, HE, false, false, TDG>(a, T, D + di, Ls, k, gpass,
                                                                     gterms, fallback);
      }
      if (fallback) return 0.0;  // the whole sample is re-evaluated in fp64
    }
    npass += gpass;
    nterms += gterms;
  } else {
    constexpr bool CY = cycle_form<ORDER, Q, false, X, false>();
    sum = diag_weight32<ORDER, Q, X, V, HE, CY, SCR, TD>(a, T, D, Ls, k, npass, nterms, fallback);
    if constexpr (SCR) return sum;
    if (fallback) return 0.0;
  }
  return jac * (x0p * x0p) * jc * sum;
}

// Kernel mode P: 0 fp64; 1 fp32 with the fp64 fallback; 2 fp64 with the
// Hartree-Fock spectrum (the fp32 integrand has the free spectrum only);
// 3 and 4: modes 0 and 1 for diagram groups (tasks of several descriptors);
// 5 and 6: fp64 with the regularised components, single diagrams / groups.
template <int P>
constexpr int prec_of() {
  return (P == 1 || P == 4) ? 1 : (P == 2 ? 2 : 0);
}
template <int P>
constexpr bool group_of() {
  return P == 3 || P == 4 || P == 6;
}
template <int P>
constexpr bool reg_of() {
  return P >= 5;
}
// Per-vertex-pair inversion (see diag_weight64) where the registers it frees
// give the kernel one more wave per SIMD: the third-order fp32 kernels (their
// fp64 re-evaluation path) fit in 168 VGPRs with it (3 waves instead of 2).
// Elsewhere the prefix form, which issues fewer instructions, at the same
// occupancy.
template <int ORDER, int Q, int P>
constexpr bool pair_inv() {
  return ORDER == 3 && prec_of<P>() == 1;
}

template <int ORDER, int Q, int P, bool X, int HE>
__device__ __forceinline__ double eval_sample(const KArgs &a, const TaskDev *__restrict__ T,
                                              const DiagDev *__restrict__ D,
                                              const SampleLds &Ls, uint64_t s,
                                              uint32_t iter, int *bins, uint32_t &npass,
                                              uint32_t &nterms, uint32_t &nfb) {
  constexpr int PP = prec_of<P>();
  constexpr bool G = group_of<P>();
  constexpr bool PI = pair_inv<ORDER, Q, P>();
  double w = 0.0;
  with_variant<ORDER, G, cycle_form<ORDER, Q, G, X, PP == 2>()>(D, [&](auto vt) {
    constexpr int V = decltype(vt)::value;
    const double jc = jac_const<ORDER, V>(a, T, D);
    if (PP != 1) {
      w = eval_fp64<ORDER, Q, PP == 2, G, X, PI, V, false, HE>(a, T, D, Ls, jc, s, iter, bins, npass, nterms);
      return;
    }
    bool fb = false;
    w = eval_fp32<ORDER, Q, G, X, V, HE>(a, T, D, Ls, jc, s, iter, bins, npass, nterms, fb);
    if (fb) {
      ++nfb;
      w = eval_fp64<ORDER, Q, false, G, X, PI, V, false, HE>(a, T, D, Ls, jc, s, iter, bins, npass, nterms);
    }
  });
  return w;
}

// Pauli screen of the sample loops in mode P: every sample first runs the
// integrand up to its Pauli test (the map, the momenta, the occupations and,
// in nuclear matter, the label cycles left open); a sample that fails adds
// its zero at once, and the others are queued per wavefront and evaluated 64
// at a time, from their random words again.  Most samples are Pauli-blocked,
// so whole wavefronts then run the denominators, interactions and label sum
// instead of wavefronts with most lanes idle.  The queued evaluation repeats
// the screen's arithmetic, so both take the same Pauli decision; a sample the
// fp32 screen finds within the fp64 band is queued, and its evaluation then
// falls back.  Fifth-order single diagrams (the free spectrum, the factorised
// label sums), where the work after the Pauli test dominates: measured on
// MI355X, nuclear matter fp32 and fp64 +25% (fp64 persistent +80%), neutron
// matter fp32 +18% and fp64 +8% (fp64 persistent -10%).  At fourth order it
// was slower (per-diagram kernels -13%, persistent -10 to -17%).
template <int ORDER, int Q, int P, bool X>
constexpr bool screen_on() {
  return ORDER >= 5 && (P == 0 || P == 1) && !X;
}

// Appends the lanes with `flag` set to a wavefront's queue in LDS (ballot
// order, so the order is deterministic); n is wave-uniform.
__device__ __forceinline__ void wave_queue_push(uint32_t *q, int &n, bool flag, uint32_t v) {
  const uint64_t mask = __ballot(flag);
  if (flag) {
    const uint32_t below = __builtin_amdgcn_mbcnt_hi(
        static_cast<uint32_t>(mask >> 32), __builtin_amdgcn_mbcnt_lo(static_cast<uint32_t>(mask), 0u));
    q[n + static_cast<int>(below)] = v;
  }
  n += __popcll(mask);
  __builtin_amdgcn_wave_barrier();
}

// Drops the first `take` entries of a wavefront's queue (take <= 64, at most
// 64 entries left behind them).
__device__ __forceinline__ void wave_queue_pop(uint32_t *q, int &n, int take, int lane) {
  __builtin_amdgcn_wave_barrier();
  const int rest = n - take;
  const uint32_t moved = (lane < rest) ? q[take + lane] : 0u;
  __builtin_amdgcn_wave_barrier();
  if (lane < rest) q[lane] = moved;
  __builtin_amdgcn_wave_barrier();
  n = rest;
}

// Bytes of the label-cycle table a sample or dump kernel of mode P holds in LDS.
template <int ORDER, int Q, int P, bool X>
constexpr size_t cycle_lds_bytes() {
  if (cycle_form<ORDER, Q, group_of<P>(), X, prec_of<P>() == 2>())
    return cycle_table_bytes<ORDER>();
  if (group_of<P>() && group_cycle_form<ORDER, Q, X, prec_of<P>() == 2>())
    return kGroupCycleTables * cycle_table_bytes<ORDER>();
  return 0;
}
template <int ORDER, int Q, int P, bool X>
constexpr bool holds_cycles() {
  return cycle_lds_bytes<ORDER, Q, P, X>() > 0;
}

// Builds the label-cycle tables of task T's diagram (one) or of its group's
// members (one per member, consecutive) at tab; the whole block takes part.
template <int ORDER, int Q, int P, bool X>
__device__ __forceinline__ void build_task_cycles(const DiagDev *__restrict__ D,
                                                  const TaskDev *__restrict__ T, void *tab) {
  if constexpr (group_of<P>()) {
    for (int di = 0; di < T->ndiag; ++di)
      build_cycle_table<ORDER>(D + di, static_cast<char *>(tab) + di * cycle_table_bytes<ORDER>());
  } else {
    build_cycle_table<ORDER>(D, tab);
  }
}

// HF spline tables held in LDS in mode P
template <int Q, int P>
constexpr int lds_tables() {
  return prec_of<P>() == 2 ? (Q == 4 ? 2 : 1) : 0;
}

// ---------------------------------------------------------------------------
// Work item: blockDim.x * spt consecutive samples of one task (HE: the
// regulator exponent's half fixed at compile time, or 0, see reg_pow)

// LDS of a sample block: turn and 2^(j/64) tables, HF tables, grid (e, width)
// pairs, histogram, reduction scratch, fp64 re-evaluation queues and Pauli
// screen queues (128 sample offsets per wavefront each), label-cycle
// table(s).
struct BlockLds {
  SampleLds Ls;
  double2 *g;
  double *h;
  double *red;
};

// Carves the block's LDS and loads the task-independent tables.
template <int ORDER, int Q, int P, bool X>
__device__ __forceinline__ void block_lds(const KArgs &a, double *smem, BlockLds &B) {
  constexpr int ND = 3 * (ORDER + 1);
  constexpr int ntab = lds_tables<Q, P>();
  SinCos *turn = reinterpret_cast<SinCos *>(smem);
  double *ex = reinterpret_cast<double *>(turn + kTurnEntries);
  double *hf = ex + kExp2Entries;
  B.g = reinterpret_cast<double2 *>(hf + hf_lds_doubles(ntab));
  B.h = reinterpret_cast<double *>(B.g + ND * a.phys.nb);
  B.red = B.h + ND * a.phys.nb;
  const int nw = blockDim.x >> 6;
  B.Ls.turn = turn;
  B.Ls.ex = ex;
  B.Ls.hf = ntab ? hf : nullptr;
  B.Ls.g = B.g;
  uint32_t *queue_end = reinterpret_cast<uint32_t *>(B.red + 6 * nw) + 256 * nw;
  B.Ls.cyc = holds_cycles<ORDER, Q, P, X>() ? queue_end : nullptr;
  load_turn_table(turn, ex);
}

// Loads task t's tables into the block's LDS: HF spline entries, grid pairs
// (e_b + w_b 2^-33, w_b), a zeroed histogram and the label-cycle table(s) of
// its diagram(s).  The caller synchronises before and after.
template <int ORDER, int Q, int P, bool X>
__device__ __forceinline__ void task_lds(const KArgs &a, int t, BlockLds &B) {
  constexpr int ND = 3 * (ORDER + 1);
  constexpr int ntab = lds_tables<Q, P>();
  const TaskDev *__restrict__ T = a.tasks + t;
  const int nb = a.phys.nb;
  const int tid = threadIdx.x, bs = blockDim.x;
  if constexpr (ntab > 0) {
    double *hf = const_cast<double *>(B.Ls.hf);
    const double *src = a.hf + 4 * static_cast<size_t>(T->hf_off);
    const int n = static_cast<int>(hf_lds_doubles(ntab));
    for (int i = tid; i < n; i += bs) hf[i] = src[i];
  }
  const double *ge = a.grids + T->grid_off;
  for (int i = tid; i < ND * nb; i += bs) {
    const int m = i / nb, b = i - m * nb;
    const double e0 = ge[m * (nb + 1) + b], e1 = ge[m * (nb + 1) + b + 1];
    B.g[i] = make_double2(fma(e1 - e0, 0x1p-33, e0), e1 - e0);
    B.h[i] = 0.0;
  }
  if constexpr (holds_cycles<ORDER, Q, P, X>())
    build_task_cycles<ORDER, Q, P, X>(a.diags + T->diag, T, const_cast<void *>(B.Ls.cyc));
}

// Adds the block's LDS histogram of task t to the task's histogram.
template <int ORDER>
__device__ __forceinline__ void hist_flush(const KArgs &a, int t, const double *h) {
  constexpr int ND = 3 * (ORDER + 1);
  double *hg = a.hists + a.tasks[t].hist_off;
  for (int i = threadIdx.x; i < ND * a.phys.nb; i += blockDim.x) {
    const double v = h[i];
    if (v != 0.0) atomicAdd(&hg[i], v);
  }
}

// The samples of one work item of task t (the task's tables in LDS): sums,
// histogram entries (LDS), and the item's partial sums and counters.
// VF: the diagram variant (see kPerItem).
template <int ORDER, int Q, int P, bool X, int HE, int VF = kPerItem>
__device__ __forceinline__ void item_samples(const KArgs &a, int t, int item, const BlockLds &B) {
  constexpr int ND = 3 * (ORDER + 1);
  const TaskDev *__restrict__ T = a.tasks + t;
  const DiagDev *__restrict__ D = a.diags + T->diag;
  const int nb = a.phys.nb;
  const int tid = threadIdx.x, bs = blockDim.x;
  const SampleLds &Ls = B.Ls;
  double *h = B.h;
  double *red = B.red;

  const uint64_t N = T->nsamples;
  const uint32_t iter = T->iter;
  const double shift = T->shift;
  const uint64_t base = static_cast<uint64_t>(item - T->item_begin) * bs * a.spt;
  double s1 = 0.0, c1 = 0.0, s2 = 0.0, c2 = 0.0;
  uint32_t npass = 0, nterms = 0, nfb = 0;
  // regularised components: sum (w_k - shift) and sum (w_k - shift)^2 with
  // the main component's shift (a thread adds at most spt terms: plain sums)
  constexpr bool R = reg_of<P>();
  double rs[R ? kRegSums : 1];
#pragma unroll
  for (int j = 0; j < (R ? kRegSums : 1); ++j) rs[j] = 0.0;
  // a thread adds at most spt terms of the shifted sums: plain sums; the
  // merges across threads and items keep the rounding errors
  auto accumulate = [&](double w, const int *bins) {
    const double d = w - shift;
    s1 += d;
    s2 = fma(d, d, s2);
    const double w2 = w * w;
    if (w2 != 0.0) {
#pragma unroll
      for (int m = 0; m < ND; ++m) atomicAdd(&h[m * nb + bins[m]], w2);
    }
  };
  // a sample that fails the Pauli screen: weight zero
  auto accumulate_zero = [&]() {
    const double d = -shift;
    s1 += d;
    s2 = fma(d, d, s2);
  };
  constexpr int PP = prec_of<P>();
  constexpr bool G = group_of<P>();
  constexpr bool PI = pair_inv<ORDER, Q, P>();
  constexpr bool SCR = screen_on<ORDER, Q, P, X>();
  const int lane = tid & 63;
  // per wavefront: the fp64 re-evaluation queue, then the Pauli screen's
  uint32_t *queue = reinterpret_cast<uint32_t *>(red + 6 * (bs >> 6)) + 128 * (tid >> 6);
  uint32_t *pqueue = queue + 128 * (bs >> 6);
  // the sample loops, specialised per diagram variant (uniform per item)
  auto loops = [&](auto vt) {
    constexpr int V = decltype(vt)::value;
    // loop coefficients from the LDS table (descriptor-driven kernels of
    // orders 4 and 5)
    // the loop coefficients decoded in the descriptor (desc_coef)
    constexpr bool TD = desc_coef<ORDER, P, VF>() && !FixedMasks<ORDER, V>::kFixed;
    const double jc = jac_const<ORDER, V>(a, T, D);
    if constexpr (SCR && PP == 0) {
      int pn = 0;  // wave-uniform
      auto drain_pass = [&](int take) {
        if (lane < take) {
          const uint64_t s = base + pqueue[lane];
          int bins[ND];
          const double w = eval_fp64<ORDER, Q, false, G, X, PI, V, false, HE, false, TD>(
              a, T, D, Ls, jc, s, iter, bins, npass, nterms);
          accumulate(w, bins);
        }
        wave_queue_pop(pqueue, pn, take, lane);
      };
      for (int kk = 0; kk < a.spt; ++kk) {
        const uint64_t s = base + static_cast<uint64_t>(kk) * bs + tid;
        bool go = false;
        if (s < N) {
          int bins[ND];
          go = eval_fp64<ORDER, Q, false, G, X, PI, V, false, HE, true, TD>(
                   a, T, D, Ls, jc, s, iter, bins, npass, nterms) != 0.0;
          if (!go) accumulate_zero();
        }
        wave_queue_push(pqueue, pn, go, static_cast<uint32_t>(s - base));
        if (pn >= 64) drain_pass(64);
      }
      while (pn > 0) drain_pass(pn < 64 ? pn : 64);
    } else if constexpr (PP != 1) {
      for (int kk = 0; kk < a.spt; ++kk) {
        const uint64_t s = base + static_cast<uint64_t>(kk) * bs + tid;
        if (s < N) {
          int bins[ND];
          if constexpr (R) {
            double wr[kMaxReg];
            const double w = eval_fp64<ORDER, Q, false, G, X, PI, V, true, HE, false, TD>(
                a, T, D, Ls, jc, s, iter, bins, npass, nterms, wr);
            accumulate(w, bins);
            // the extrapolation's weights sum to one, so its shifted value
            // is the weighted sum of the components' shifted values
            double dx = 0.0;
#pragma unroll
            for (int r = 0; r < kMaxReg; ++r) {
              const double d = wr[r] - shift;
              rs[2 * r] += d;
              rs[2 * r + 1] += d * d;
              dx = fma(a.reg_coef[r], d, dx);
            }
            rs[2 * kMaxReg] += dx;
            rs[2 * kMaxReg + 1] += dx * dx;
          } else {
            const double w = eval_fp64<ORDER, Q, PP == 2, G, X, PI, V, false, HE, false, TD>(
                a, T, D, Ls, jc, s, iter, bins, npass, nterms);
            accumulate(w, bins);
          }
        }
      }
    } else {
      // fp32 pass; samples in the fp64 band are queued per wavefront (ballot
      // order, so the accumulation order is deterministic) and re-evaluated in
      // fp64 by whole wavefronts, 64 at a time
      int qn = 0;  // wave-uniform
      auto drain = [&](int take) {
        if (lane < take) {
          const uint64_t s = base + queue[lane];
          int bins[ND];
          const double w = eval_fp64<ORDER, Q, false, G, X, PI, V, false, HE, false, TD>(
              a, T, D, Ls, jc, s, iter, bins, npass, nterms);
          accumulate(w, bins);
        }
        __builtin_amdgcn_wave_barrier();
        const int rest = qn - take;
        uint32_t moved = (lane < rest) ? queue[take + lane] : 0u;
        __builtin_amdgcn_wave_barrier();
        if (lane < rest) queue[lane] = moved;
        __builtin_amdgcn_wave_barrier();
        qn = rest;
      };
      if constexpr (SCR) {
        int pn = 0;  // wave-uniform
        auto drain_pass = [&](int take) {
          bool fb = false;
          uint32_t off = 0u;
          if (lane < take) {
            off = pqueue[lane];
            int bins[ND];
            const double w = eval_fp32<ORDER, Q, G, X, V, HE, false, TD>(
                a, T, D, Ls, jc, base + off, iter, bins, npass, nterms, fb);
            if (!fb) accumulate(w, bins);
          }
          if (fb) ++nfb;
          wave_queue_push(queue, qn, fb, off);
          wave_queue_pop(pqueue, pn, take, lane);
          if (qn >= 64) drain(64);
        };
        for (int kk = 0; kk < a.spt; ++kk) {
          const uint64_t s = base + static_cast<uint64_t>(kk) * bs + tid;
          bool go = false;
          if (s < N) {
            int bins[ND];
            bool unused = false;
            go = eval_fp32<ORDER, Q, G, X, V, HE, true, TD>(a, T, D, Ls, jc, s, iter, bins,
                                                                 npass, nterms, unused) != 0.0;
            if (!go) accumulate_zero();
          }
          wave_queue_push(pqueue, pn, go, static_cast<uint32_t>(s - base));
          if (pn >= 64) drain_pass(64);
        }
        while (pn > 0) drain_pass(pn < 64 ? pn : 64);
      } else {
        for (int kk = 0; kk < a.spt; ++kk) {
          const uint64_t s = base + static_cast<uint64_t>(kk) * bs + tid;
          bool fb = false;
          if (s < N) {
            int bins[ND];
            const double w = eval_fp32<ORDER, Q, G, X, V, HE, false, TD>(
                a, T, D, Ls, jc, s, iter, bins, npass, nterms, fb);
            if (!fb) accumulate(w, bins);
          }
          const uint64_t mask = __ballot(fb);
          if (fb) {
            const int pos = qn + __builtin_amdgcn_mbcnt_hi(
                                     static_cast<uint32_t>(mask >> 32),
                                     __builtin_amdgcn_mbcnt_lo(static_cast<uint32_t>(mask), 0u));
            queue[pos] = static_cast<uint32_t>(s - base);
            ++nfb;
          }
          qn += __popcll(mask);
          __builtin_amdgcn_wave_barrier();
          if (qn >= 64) drain(64);
        }
      }
      while (qn > 0) drain(qn < 64 ? qn : 64);
    }
  };
  if constexpr (VF >= 0) loops(std::integral_constant<int, VF>{});
  else with_variant<ORDER, G, cycle_form<ORDER, Q, G, X, PP == 2>()>(D, loops);
  // wavefront butterfly, then waves in order (compensated pairs s + c)
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) {
    const double os1 = __shfl_xor(s1, off, 64), oc1 = __shfl_xor(c1, off, 64);
    const double os2 = __shfl_xor(s2, off, 64), oc2 = __shfl_xor(c2, off, 64);
    pair_merge(s1, c1, os1, oc1);
    pair_merge(s2, c2, os2, oc2);
    npass += __shfl_xor(npass, off, 64);
    nterms += __shfl_xor(nterms, off, 64);
    nfb += __shfl_xor(nfb, off, 64);
    if constexpr (R) {
#pragma unroll
      for (int j = 0; j < kRegSums; ++j) rs[j] += __shfl_xor(rs[j], off, 64);
    }
  }
  const int wave = tid >> 6;
  uint32_t *ured = reinterpret_cast<uint32_t *>(red + 4 * (bs >> 6));
  // component sums per wave in the (fp64-only, so unused) re-evaluation queue
  double *rred = red + 6 * (bs >> 6);
  if constexpr (R) {
    if (lane == 0) {
#pragma unroll
      for (int j = 0; j < kRegSums; ++j) rred[kRegSums * wave + j] = rs[j];
    }
  }
  if (lane == 0) {
    red[4 * wave + 0] = s1;
    red[4 * wave + 1] = c1;
    red[4 * wave + 2] = s2;
    red[4 * wave + 3] = c2;
    ured[3 * wave] = npass;
    ured[3 * wave + 1] = nterms;
    ured[3 * wave + 2] = nfb;
  }
  __syncthreads();
  if (tid == 0) {
    double S1 = red[0], C1 = red[1], S2 = red[2], C2 = red[3];
    uint64_t P1 = ured[0], P2 = ured[1], P0 = ured[2];
    for (int w = 1; w < (bs >> 6); ++w) {
      pair_merge(S1, C1, red[4 * w + 0], red[4 * w + 1]);
      pair_merge(S2, C2, red[4 * w + 2], red[4 * w + 3]);
      P1 += ured[3 * w];
      P2 += ured[3 * w + 1];
      P0 += ured[3 * w + 2];
    }
    const size_t store = static_cast<size_t>(T->store_begin) + (item - T->item_begin);
    double *part = a.partials + 4 * store;
    part[0] = S1;
    part[1] = C1;
    part[2] = S2;
    part[3] = C2;
    uint64_t *K = a.counters + kItemCounters * store;
    K[0] = P0;
    K[1] = P1;
    K[2] = P2;
    if constexpr (R) {
      double *cp = a.cpart + kRegSums * store;
      for (int j = 0; j < kRegSums; ++j) {
        double v = rred[j];
        for (int w = 1; w < (bs >> 6); ++w) v += rred[kRegSums * w + j];
        cp[j] = v;
      }
    }
  }
}

// One work item with its own setup and histogram merge.
template <int ORDER, int Q, int P, bool X, int HE, int VF = kPerItem>
__device__ __forceinline__ void process_item(const KArgs &a, int t, int item, double *smem) {
  BlockLds B;
  block_lds<ORDER, Q, P, X>(a, smem, B);
  task_lds<ORDER, Q, P, X>(a, t, B);
  __syncthreads();
  item_samples<ORDER, Q, P, X, HE, VF>(a, t, item, B);
  __syncthreads();
  hist_flush<ORDER>(a, t, B.h);
}

// Waves per SIMD the sample kernels ask the compiler for (it then holds them
// within 512 / waves VGPRs, spilling the rest), as measured on MI355X:
// - fourth order: fp64, fp32, group and regularised kernels run 4-30% faster
//   at 3 waves (100-200 spilled bytes per thread) than at 2 without spills;
//   the regularised group kernel gains at 2;
// - fifth order: fp32, group and explicit-list kernels gain at 3 waves; the
//   fp64 polynomial kernel (about 360 spilled bytes at 3) and the regularised
//   single-diagram kernel are faster at their natural occupancy; the
//   regularised group kernel stays within 256 VGPRs at 2;
// - HF kernels (isospin-dependent spectra keep per-line energy differences
//   live): 2 waves from third order on, 20-45% faster than at one, except
//   fifth-order neutron matter, which loses a third to ~520 spilled bytes.
// - third order, fp64 and fp32 (single diagrams specialised per diagram):
//   4 waves with 60-130 spilled bytes beat 3 waves without (4-7%);
// - nuclear matter with the cycle form of the label sum (single diagrams,
//   work items of up to 65536 samples): fourth-order fp32 at 4 waves beats 3
//   by 1-6%; fourth-order fp64, with the loop coefficients from the
//   descriptor, runs 4% faster at 3 waves than at 4; fourth-order nuclear
//   group kernels, whose per-member cycle tables leave LDS for 3 blocks per
//   CU, run 3-5% faster at 3 waves than at 4 and 8-13% faster than at 2;
// - fifth-order nuclear matter with the Pauli screen: fp32 at 3 waves beats 4
//   by 8% and 2 by 11%, fp64 at 3 beats 2 by 11% and 4 by 16%.
// Other kernels fit their natural occupancy.
template <int ORDER, int Q, int P, bool X>
constexpr int min_waves() {
  if (P == 2) {
    if (ORDER == 2) return 3;
    if (ORDER == 3 || ORDER == 4) return 2;
    return (ORDER == 5 && Q == 4) ? 2 : 1;
  }
  if (Q == 4 && !X && (P == 0 || P == 1)) {
    if (ORDER == 4) return P == 1 ? 4 : 3;
    if (ORDER == 5) return 3;
  }
  if (ORDER == 3 && (P == 0 || P == 1)) return 4;
  if (ORDER == 4) return (P == 0 || P == 1 || P == 3 || P == 4 || P == 5) ? 3 : 2;
  if (ORDER == 5) {
    if (P == 1 || P == 3 || P == 4 || (P == 0 && X)) return 3;
    return P == 6 ? 2 : 1;
  }
  return 1;
}

// Waves per SIMD of the persistent kernels: their item loop leaves more
// registers live than a one-item kernel, and at the one-item kernels'
// occupancy the nuclear-matter kernels of orders 4 and 5 spilled 180-600
// bytes per lane.  Measured on MI355X (every third fourth-order diagram and
// every 42nd fifth-order one at the 15 nuclear-matter points, 2^22 samples
// per task): fourth order fp32 23.6 Gevals/s at 3 waves against 20.3 at 4,
// fp64 21.5 at 2 against 11.9 at 4; fifth order fp32 13.0 at 2 against 3.9 at
// 4, fp64 7.4 at 2 against 5.6 at 3.
template <int ORDER, int Q, int P, bool X>
constexpr int persistent_waves() {
  if (Q == 4 && !X && (P == 0 || P == 1)) {
    if (ORDER == 4) return P == 1 ? 3 : 2;
    if (ORDER == 5) return 2;
  }
  return min_waves<ORDER, Q, P, X>();
}

// One task per launch: block b processes work item item_begin + b.
template <int ORDER, int Q, int P, bool X, int HE>
__global__ __launch_bounds__(256, (min_waves<ORDER, Q, P, X>())) void sample_single(KArgs a, int t) {
  extern __shared__ double smem[];
  process_item<ORDER, Q, P, X, HE>(a, t, a.tasks[t].item_begin + blockIdx.x, smem);
}

// One launch over the work items of the tasks of one order: olist[k0, k1)
// lists them as (first item, task) with ascending first item, their items are
// numbered contiguously from olist[k0].x, and block b takes item
// olist[k0].x + b.  One launch per order keeps each launch's register
// allocation that of its own order.
template <int ORDER, int Q, int P, bool X, int HE>
__global__ __launch_bounds__(256, (min_waves<ORDER, Q, P, X>())) void sample_order(KArgs a, int k0, int k1) {
  extern __shared__ double smem[];
  const int2 *__restrict__ ol = a.olist;
  const int item = ol[k0].x + static_cast<int>(blockIdx.x);
  int lo = k0, hi = k1 - 1;  // last entry with first item <= item
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (ol[mid].x <= item) lo = mid;
    else hi = mid - 1;
  }
  process_item<ORDER, Q, P, X, HE>(a, ol[lo].y, item, smem);
}

// sample_order for the tasks of one diagram whose descriptor masks and label
// cycles are compile-time constants (FixedMasks<ORDER, V>, V = the diagram
// id): the loop-momentum sums keep only their nonzero terms and need no
// scalar decoding, and the cycle words take no scalar registers.  The same
// operations as the descriptor-driven kernel (a product with a coefficient 0,
// +-1, +-2 or +-1/2 is exact), but with the masks known the compiler may fuse
// other multiply-adds (shared vertex momenta), so the weights agree to their
// last bits.  Built for 3 waves per SIMD, as measured on the 585
// fourth-order nuclear-matter tasks: fp64 44.1 Gevals/s at 3 against 36.6 at
// 4 and 44.1 at 2; fp32 47.6 at 3 against 41.0 at 2 and 49.5 at 4, where 31
// spilled VGPRs raise the HBM traffic from 1.1 GB to 17 GB per iteration.
template <int ORDER, int Q, int P, int HE, int V>
__global__ __launch_bounds__(256, 3) void sample_order_fixed(
    KArgs a, int k0, int k1) {
  static_assert(FixedMasks<ORDER, V>::kFixed, "a per-diagram kernel needs the diagram's masks");
  extern __shared__ double smem[];
  const int2 *__restrict__ ol = a.olist;
  const int item = ol[k0].x + static_cast<int>(blockIdx.x);
  int lo = k0, hi = k1 - 1;  // last entry with first item <= item
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (ol[mid].x <= item) lo = mid;
    else hi = mid - 1;
  }
  process_item<ORDER, Q, P, false, HE, V>(a, ol[lo].y, item, smem);
}

// Persistent launch over the work items of the tasks of one order (as
// sample_order, nitems items from olist[k0].x on): a grid of about as many
// blocks as are resident on the device at once; each block claims chunks of
// `chunk` consecutive items from the order's counter a.queue[ORDER] until all
// are taken.  Claims ascend, so a block meets the tasks in ascending order:
// it keeps the current task's grid, histogram and label-cycle table in LDS
// across that task's items and merges the histogram into the task's once per
// run of items (instead of once per item).  The counter starts at zero (task
// set initialisation) and the iteration end zeroes it for the next iteration.
template <int ORDER, int Q, int P, bool X, int HE>
__global__ __launch_bounds__(256, (persistent_waves<ORDER, Q, P, X>())) void sample_persistent(
    KArgs a, int k0, int k1, int nitems, int chunk) {
  extern __shared__ double smem[];
  __shared__ int claim;
  const int2 *__restrict__ ol = a.olist;
  const int first = ol[k0].x;
  BlockLds B;
  block_lds<ORDER, Q, P, X>(a, smem, B);
  int cur = -1, lo = k0;
  for (;;) {
    __syncthreads();  // every thread has read the previous claim
    if (threadIdx.x == 0) claim = atomicAdd(a.queue + ORDER, chunk);
    __syncthreads();
    const int c0 = claim;
    if (c0 >= nitems) break;
    const int c1 = min(c0 + chunk, nitems);
    for (int k = c0; k < c1; ++k) {
      const int item = first + k;
      while (lo + 1 < k1 && ol[lo + 1].x <= item) ++lo;
      const int t = ol[lo].y;
      __syncthreads();  // the previous item's reduction scratch has been read
      if (t != cur) {
        if (cur >= 0) hist_flush<ORDER>(a, cur, B.h);
        __syncthreads();
        task_lds<ORDER, Q, P, X>(a, t, B);
        __syncthreads();
        cur = t;
      }
      // opaque to the optimiser: nothing of one item's evaluation is kept
      // live into the next (the body then has the registers of a one-item
      // kernel)
      int tt = t, ii = item;
      asm volatile("" : "+s"(tt), "+s"(ii));
      item_samples<ORDER, Q, P, X, HE>(a, tt, ii, B);
    }
  }
  __syncthreads();
  if (cur >= 0) hist_flush<ORDER>(a, cur, B.h);
}

// ---------------------------------------------------------------------------
// Per-sample dump for parity checks: thread i evaluates sample first + i.

// Regularised modes: out_reg (if not null) receives the components,
// out_reg[i * nreg + k] for component k + 1.
template <int ORDER, int Q, int P, bool X, int HE>
__global__ __launch_bounds__(256) void dump_samples(KArgs a, int t, uint32_t iter, uint64_t first,
                                                   uint64_t count, double *out, double *out_reg) {
  extern __shared__ double smem[];
  constexpr int ND = 3 * (ORDER + 1);
  constexpr bool PI = pair_inv<ORDER, Q, P>();
  const TaskDev *T = a.tasks + t;
  const DiagDev *D = a.diags + T->diag;
  const int nb = a.phys.nb;
  SampleLds Ls;
  double2 *g;
  carve_lds(a, T, lds_tables<Q, P>(), ND, smem, Ls, g);
  const double *ge = a.grids + T->grid_off;
  for (int i = threadIdx.x; i < ND * nb; i += blockDim.x) {
    const int m = i / nb, b = i - m * nb;
    const double e0 = ge[m * (nb + 1) + b], e1 = ge[m * (nb + 1) + b + 1];
    g[i] = make_double2(fma(e1 - e0, 0x1p-33, e0), e1 - e0);
  }
  if constexpr (holds_cycles<ORDER, Q, P, X>()) {
    void *tab = g + ND * nb;
    build_task_cycles<ORDER, Q, P, X>(D, T, tab);
    Ls.cyc = tab;
  }
  __syncthreads();
  const uint64_t i = static_cast<uint64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < count) {
    int bins[ND];
    uint32_t np = 0, nt = 0, nf = 0;
    if constexpr (reg_of<P>()) {
      double wr[kMaxReg];
      with_variant<ORDER, group_of<P>(), cycle_form<ORDER, Q, group_of<P>(), X, false>()>(
          D, [&](auto vt) {
        constexpr int V = decltype(vt)::value;
        out[i] = eval_fp64<ORDER, Q, false, group_of<P>(), X, PI, V, true, HE>(
            a, T, D, Ls, jac_const<ORDER, V>(a, T, D), first + i, iter, bins, np, nt, wr);
      });
      if (out_reg)
        for (int r = 0; r < a.nreg; ++r) out_reg[i * a.nreg + r] = wr[r];
    } else {
      out[i] = eval_sample<ORDER, Q, P, X, HE>(a, T, D, Ls, first + i, iter, bins, np, nt, nf);
    }
  }
}

// Mode of a sample kernel from the precision, spectrum, regularisation and
// grouping (see prec_of, group_of, reg_of); -1 if no kernel exists: the HF
// spectrum runs the fp64 integrand (mode 2) whatever the precision, the
// regularised components the fp64 integrand (modes 5, 6) with the free
// spectrum.
__host__ inline int mode_of(const KArgs &a, int prec, bool group) {
  if (a.nreg > 0) return a.phys.spectrum ? -1 : 5 + (group ? 1 : 0);
  if (a.phys.spectrum) return group ? -1 : 2;  // HF groups are not built
  return (prec ? 1 : 0) + (group ? 3 : 0);
}

}  // namespace mbpt
