// Host runtime and C ABI of the MI355X VEGAS library for MBPT energy
// diagrams.  See include/mbpt_vegas.h for the contract of every entry point.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstddef>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <tuple>
#include <utility>
#include <vector>

#include "diagrams.hpp"
#include "device_types.hpp"
#include "kernels.hpp"
#include "mbpt_vegas.h"
#include "runtime.hpp"

using namespace mbpt;

namespace mbpt {

void set_err(mbpt_context *ctx, const std::string &msg) {
  if (ctx) ctx->err = msg;
}

int hip_fail(mbpt_context *ctx, hipError_t e, const char *what) {
  set_err(ctx, std::string(what) + ": " + hipGetErrorString(e));
  return MBPT_EHIP;
}

#define HIPCHK(ctx, call)                                \
  do {                                                   \
    hipError_t e_ = (call);                              \
    if (e_ != hipSuccess) return hip_fail(ctx, e_, #call); \
  } while (0)

static size_t align256(size_t x) { return (x + 255) & ~static_cast<size_t>(255); }

// Algorithmic FLOPs of one evaluation, counted from the descriptor:
// FMA = 2, add/mul = 1, each exp / sqrt / sin / cos / division = 1 (also
// tallied separately).  Split into the part every sample needs (map, loop
// momenta, line momenta, Pauli tests), the part a sample past the Pauli test
// needs (denominators, matrix elements, weight, accumulation) and the part
// per label term evaluated.
void count_flops(const Diagram &d, int q, int half_exp, int label_mode, int spectrum,
                 FlopModel &f) {
  const int n = d.order, L = d.nloops, NL = d.nlines, NC = d.ncuts, ND = d.ndim;
  const int H = n / 2;
  double pre = 0, pre_t = 0;
  pre += 6.0 * ND;                  // bin fraction (2), x = e + r w (2), jacobian (2)
  pre += 13.0 * L;                  // radius, cos, sin theta, k components, jacobian
  pre_t += 3.0 * L;                 // sqrt, sin, cos
  for (int l = 0; l < NL; ++l) {
    int nnz = 0;
    for (int j = 0; j < L; ++j) nnz += d.coef[l][j] != 0;
    pre += 3.0 * std::max(0, nnz - 1);  // tree-line sums
    pre += 5.0 + 1.0;                    // k^2, eps
    pre += (q == 4) ? 2.0 : 1.0;         // occupation tests
    if (spectrum) {
      pre_t += 1.0;                      // |k|
      pre += 8.0 * (q == 4 ? 2 : 1) + 1; // spline(s) and their sum / difference
    }
  }
  double post = 0, post_t = 0;
  for (int c = 0; c < NC; ++c) {
    int nnz = 0;
    for (int l = 0; l < NL; ++l) nnz += d.cut[c][l] != 0;
    post += nnz - 1;
  }
  post += std::max(0, NC - 1);  // product of denominators
  // per vertex: p, p' (6 + 6), p^2, p'^2, p.p' (15), powers, exponent (2),
  // q^2 +- (4 + 2), C0 + (2), regulator products (2), V_d - V_e (1)
  post += n * (6 + 6 + 15 + 2.0 * (half_exp - 1) + 2 + 6 + 2 + 2 + 1);
  post_t += n * 3.0;            // exp and two divisions
  post += 3.0;                  // weight: jacobian * prefactor * label sum
  post_t += 1.0;                // one division by the denominators
  post_t += (NC == 0) ? -1.0 : 0.0;
  // HF in nuclear matter: per isospin configuration its own denominators
  // (2 per line of each cut, their product) and one division
  const double iso_den = (spectrum && q == 4) ? 2.0 * NC * NL + NC + 1.0 : 0.0;
  if (label_mode) {
    f.per_term = n + 1.0;       // explicit term: product of n factors, multiply-add
  } else {
    // factorised: monomial tables of the two vertex halves (2^H + 2^{n-H}
    // products) once per sample, then per isospin group 2^n + 2^{n-H} FMAs
    post += (1 << H) + (1 << (n - H)) - 2;
    f.per_term = 2.0 * ((1 << n) + (1 << (n - H))) + iso_den;
  }
  double acc = 4.0 + 1.0 + ND;  // shifted sums (d = w - c, s1 += d, s2 += d^2), w^2, histogram adds
  f.pre = pre + pre_t + acc;    // every sample is accumulated
  // map, loop momenta and accumulation: once per sample even for a group
  f.transc_shared = 3.0 * L;
  f.shared = 6.0 * ND + 13.0 * L + f.transc_shared + acc;
  f.post = post + post_t;
  f.all_units = 0.0;
  f.transc_pre = pre_t;
  f.transc_post = post_t;
}

}  // namespace mbpt

// ---------------------------------------------------------------------------
// Context

extern "C" int mbpt_context_create(const mbpt_context_desc *desc, mbpt_context **out) {
  if (!out) return MBPT_EINVAL;
  *out = nullptr;
  mbpt_context_desc d{};
  d.device = 0;
  d.stream = nullptr;
  d.precision = MBPT_FP64;
  d.seed = 1;
  d.n_bins = 50;
  d.alpha = 1.5;
  d.kcut_extra = 3.0;
  d.fp32_band_k = 1e-4;
  d.fp32_band_d = 1e-2;
  d.label_mode = 0;
  d.spectrum = MBPT_SPECTRUM_FREE;
  if (desc) d = *desc;
  if (d.n_bins < 2 || d.n_bins > kMaxBins || !(d.alpha > 0.0) || !(d.kcut_extra >= 0.0) ||
      (d.precision != MBPT_FP64 && d.precision != MBPT_FP32) || d.fp32_band_k < 0.0 ||
      d.fp32_band_d < 0.0 || (d.label_mode != 0 && d.label_mode != 1) ||
      (d.spectrum != MBPT_SPECTRUM_FREE && d.spectrum != MBPT_SPECTRUM_HF))
    return MBPT_EINVAL;
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || d.device < 0 || d.device >= ndev) return MBPT_EHIP;
  if (hipSetDevice(d.device) != hipSuccess) return MBPT_EHIP;
  auto *ctx = new mbpt_context();
  ctx->desc = d;
  ctx->stream = static_cast<hipStream_t>(d.stream);
  ctx->v = mbpt_interaction{-1.0, -2.0, 0.7, 2.0, 4, 41.47, 197.3269804};
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, d.device) == hipSuccess) ctx->num_cus = prop.multiProcessorCount;
  *out = ctx;
  return MBPT_OK;
}

extern "C" void mbpt_context_destroy(mbpt_context *ctx) {
  if (!ctx) return;
  for (auto &ev : ctx->events) {
    (void)hipEventDestroy(ev.first);
    (void)hipEventDestroy(ev.second);
  }
  delete ctx;
}

extern "C" const char *mbpt_last_error(const mbpt_context *ctx) {
  return ctx ? ctx->err.c_str() : "null context";
}

extern "C" int mbpt_set_interaction(mbpt_context *ctx, const mbpt_interaction *v) {
  if (!ctx || !v) return MBPT_EINVAL;
  if (v->reg_exp < 2 || v->reg_exp > 16 || (v->reg_exp & 1) || !(v->Lambda > 0) ||
      !(v->hbar2_m > 0) || !(v->hbarc > 0) || !(v->mpi > 0)) {
    set_err(ctx, "mbpt_set_interaction: invalid interaction parameters");
    return MBPT_EINVAL;
  }
  ctx->v = *v;
  ++ctx->epoch;
  return MBPT_OK;
}

extern "C" int mbpt_set_spectrum(mbpt_context *ctx, int spectrum) {
  if (!ctx || (spectrum != MBPT_SPECTRUM_FREE && spectrum != MBPT_SPECTRUM_HF)) return MBPT_EINVAL;
  ctx->desc.spectrum = spectrum;
  ++ctx->epoch;
  return MBPT_OK;
}

extern "C" int mbpt_set_regularization(mbpt_context *ctx, int n_eta, double eta) {
  if (!ctx) return MBPT_EINVAL;
  if (n_eta < 0 || n_eta > kMaxReg || (n_eta > 0 && !(eta > 0.0 && std::isfinite(eta)))) {
    set_err(ctx, "set_regularization: n_eta must be 0..4 and eta > 0");
    return MBPT_EINVAL;
  }
  ctx->reg_n = n_eta;
  ctx->reg_eta = n_eta > 0 ? eta : 0.0;
  ++ctx->epoch;
  return MBPT_OK;
}

extern "C" int mbpt_set_fp32_target(mbpt_context *ctx, double rel) {
  if (!ctx || !(rel >= 0.0) || !std::isfinite(rel)) return MBPT_EINVAL;
  ctx->fp32_rel_target = rel;
  ++ctx->epoch;
  return MBPT_OK;
}

extern "C" int mbpt_set_precision(mbpt_context *ctx, int precision) {
  if (!ctx || (precision != MBPT_FP64 && precision != MBPT_FP32)) return MBPT_EINVAL;
  ctx->desc.precision = precision;
  ++ctx->epoch;
  return MBPT_OK;
}

// ---------------------------------------------------------------------------
// Generator queries

extern "C" int mbpt_num_diagrams(int order, int *count) {
  if (!count) return MBPT_EINVAL;
  const int n = num_diagrams(order);
  if (n < 0) return MBPT_EINVAL;
  *count = n;
  return MBPT_OK;
}

extern "C" int mbpt_diagram_matrix(int order, int id, int *M, double *prefactor) {
  const Diagram *d = get_diagram(order, id);
  if (!d || !M) return MBPT_EINVAL;
  for (int u = 0; u < order; ++u)
    for (int v = 0; v < order; ++v) M[u * order + v] = d->M[u][v];
  if (prefactor) *prefactor = d->prefactor;
  return MBPT_OK;
}

extern "C" int mbpt_diagram_label_stats(int order, int id, int matter, int *n_assign,
                                        int *n_isospin, int *n_terms) {
  const Diagram *d = get_diagram(order, id);
  if (!d || (matter != MBPT_NEUTRON && matter != MBPT_NUCLEAR)) return MBPT_EINVAL;
  const LabelList ll = build_labels(*d, matter == MBPT_NUCLEAR ? 4 : 2);
  if (n_assign) *n_assign = ll.n_assign;
  if (n_isospin) *n_isospin = ll.n_isospin;
  if (n_terms) *n_terms = static_cast<int>(ll.terms.size());
  return MBPT_OK;
}

extern "C" int mbpt_group_members(int order, int p, int *ids, int cap, int *n) {
  if (!n || order < 1 || order > kMaxOrder || p < 0 || cap < 0) return MBPT_EINVAL;
  const std::vector<int> m = group_members(order, p);
  *n = static_cast<int>(m.size());
  if (ids)
    for (int i = 0; i < *n && i < cap; ++i) ids[i] = m[i];
  return MBPT_OK;
}

extern "C" int mbpt_diagram_label_poly(int order, int id, int matter, double *coef, int max_rows,
                                       int *n_rows) {
  const Diagram *d = get_diagram(order, id);
  if (!d || !n_rows || (matter != MBPT_NEUTRON && matter != MBPT_NUCLEAR)) return MBPT_EINVAL;
  const LabelTables lt = label_tables(*d, matter == MBPT_NUCLEAR ? 4 : 2);
  *n_rows = static_cast<int>(lt.groups.size());
  if (!coef) return MBPT_OK;
  if (*n_rows > max_rows) return MBPT_ENOMEM;
  const size_t nE = size_t{1} << order;
  for (size_t g = 0; g < lt.groups.size(); ++g)
    std::copy(lt.groups[g].coef.begin(), lt.groups[g].coef.end(), coef + g * nE);
  return MBPT_OK;
}

// ---------------------------------------------------------------------------
// Task sets

namespace mbpt {

// Descriptor fields derived from the diagram alone (loop radii, masks in
// line-slot order, prefactor with the (2 pi)^{-3L} measure).  canonical: the
// loops in the group-canonical order (particle loops first).
void fill_diag_dev(const Diagram &d, DiagDev &dd, bool canonical) {
  int slot_line[kMaxLines], canon[kMaxLoops], pos[kMaxLoops];
  line_slots(d, slot_line, canonical);
  for (int j = 0; j < d.nloops; ++j) canon[j] = j;
  if (canonical) canonical_loops(d, canon);
  for (int c = 0; c < d.nloops; ++c) pos[canon[c]] = c;
  for (int c = 0; c < d.nloops; ++c) dd.loop_part[c] = d.particle[d.loop_line[canon[c]]] ? 1 : 0;
  dd.part_mask = 0;
  for (int sl = 0; sl < d.nlines; ++sl)
    if (d.particle[slot_line[sl]]) dd.part_mask |= 1u << sl;
  dd.line_mask = (1u << d.nlines) - 1u;
  dd.pref = d.prefactor * std::pow(2.0 * M_PI, -3.0 * d.nloops);
  // coefficient of the diagram's loop j goes to bit pos[j]
  auto pack = [&](const int *c) {
    uint32_t m = 0;
    for (int j = 0; j < d.nloops; ++j) {
      const int b = pos[j];
      if (c[j] == 1) m |= 1u << b;
      else if (c[j] == -1) m |= 1u << (8 + b);
      else if (c[j] == 2) m |= 1u << (16 + b);
      else if (c[j] == -2) m |= 1u << (24 + b);
    }
    return m;
  };
  for (int sl = 0; sl < d.nlines; ++sl) dd.lmask[sl] = pack(d.coef[slot_line[sl]]);
  for (int v = 0; v < d.order; ++v) {
    int cp[kMaxLoops], cq[kMaxLoops];
    for (int j = 0; j < d.nloops; ++j) {
      cp[j] = d.coef[d.vout[v][0]][j] - d.coef[d.vout[v][1]][j];
      cq[j] = d.coef[d.vin[v][0]][j] - d.coef[d.vin[v][1]][j];
    }
    dd.pmask_v[v] = pack(cp);
    dd.qmask_v[v] = pack(cq);
  }
  for (int c = 0; c < d.ncuts; ++c)
    for (int sl = 0; sl < d.nlines; ++sl) {
      const int l = slot_line[sl];
      if (d.cut[c][l] > 0) dd.cut_hole[c] |= 1u << sl;
      if (d.cut[c][l] < 0) dd.cut_part[c] |= 1u << sl;
    }
  // the masks decoded: bit j +1, 8 + j -1, 16 + j +2, 24 + j -2 (halved
  // for the vertex sums)
  auto unpack = [&](uint32_t m, double scale, int s) {
    for (int j = 0; j < kDescCoefStride; ++j) {
      double c = 0.0;
      if (j < 8) {
        if (m & (1u << j)) c = 1.0;
        if (m & (1u << (8 + j))) c = -1.0;
        if (m & (1u << (16 + j))) c = 2.0;
        if (m & (1u << (24 + j))) c = -2.0;
      }
      dd.coef_d[s][j] = c * scale;
      dd.coef_f[s][j] = static_cast<float>(c * scale);
    }
  };
  for (int s = 0; s < kDescCoefSums; ++s)
    for (int j = 0; j < kDescCoefStride; ++j) dd.coef_d[s][j] = dd.coef_f[s][j] = 0;
  const int nl = 2 * d.order;
  for (int sl = 0; sl < nl && sl < d.nlines; ++sl) unpack(dd.lmask[sl], 1.0, sl);
  for (int v = 0; v < d.order; ++v) {
    unpack(dd.pmask_v[v], 0.5, nl + 2 * v);
    unpack(dd.qmask_v[v], 0.5, nl + 2 * v + 1);
  }
}

// The kernels of orders 1-3 take the descriptor masks of the order's
// diagrams as compile-time constants (FixedMasks); true if the generator's
// descriptors are those (checked once; order-3 group tasks take the generic
// path, so only the plain loop order is checked there).
template <int ORDER, int V>
static bool fixed_masks_match(const DiagDev &dd) {
  using F = FixedMasks<ORDER, V>;
  constexpr int NL = 2 * ORDER, L = ORDER + 1, NC = ORDER - 1;
  bool ok = dd.line_mask == F::line_mask && dd.part_mask == F::part_mask;
  for (int l = 0; l < NL; ++l) ok = ok && dd.lmask[l] == F::lmask[l];
  for (int v = 0; v < ORDER; ++v)
    ok = ok && dd.pmask_v[v] == F::pmask_v[v] && dd.qmask_v[v] == F::qmask_v[v];
  for (int c = 0; c < NC; ++c)
    ok = ok && dd.cut_hole[c] == F::cut_hole[c] && dd.cut_part[c] == F::cut_part[c];
  for (int j = 0; j < L; ++j) ok = ok && dd.loop_part[j] == F::loop_part[j];
  return ok;
}

// The tables of orders 2-4 also fix the label cycles per vertex-term choice
// (plain loop order: the single-diagram kernels).
template <int ORDER, int V>
static bool fixed_cycles_match(const Diagram &d) {
  using F = FixedMasks<ORDER, V>;
  constexpr int NE = 1 << ORDER;
  const CycleTables ct = cycle_tables(d, false);
  if (ct.masks.size() > 24 || ct.of_e.size() != static_cast<size_t>(NE)) return false;
  bool ok = true;
  for (int E = 0; E < NE; ++E)
    ok = ok && F::cyc_e32[E] ==
                   static_cast<uint32_t>(ct.of_e[E] | static_cast<uint64_t>(ct.n_of_e[E]) << 24);
  return ok;
}

// The tables of orders 1-3 also fix the neutron-matter label coefficients:
// one isospin configuration (all neutrons).
template <int ORDER, int V>
static bool fixed_labels_match(const Diagram &d, bool canonical) {
  using F = FixedMasks<ORDER, V>;
  const LabelTables lt = label_tables(d, 2, canonical);
  if (lt.groups.size() != 1 || lt.groups[0].tau != 0u ||
      lt.groups[0].coef.size() != (size_t{1} << ORDER))
    return false;
  bool ok = true;
  for (int i = 0; i < (1 << ORDER); ++i) ok = ok && lt.groups[0].coef[i] == F::label_coef_q2[i];
  return ok;
}

template <typename Dev, int... I>
static bool fixed4_match(Dev &&dev, std::integer_sequence<int, I...>) {
  return ((fixed_masks_match<4, I>(dev(4, I, false)) &&
           fixed_cycles_match<4, I>(*get_diagram(4, I))) && ...);
}

bool fixed_masks_ok() {
  static const bool ok = [] {
    bool r = true;
    auto dev = [](int order, int id, bool canonical) {
      DiagDev d{};
      fill_diag_dev(*get_diagram(order, id), d, canonical);
      return d;
    };
    for (int canonical = 0; canonical < 2; ++canonical) {
      r = r && fixed_masks_match<1, 0>(dev(1, 0, canonical != 0));
      r = r && fixed_masks_match<2, 0>(dev(2, 0, canonical != 0));
    }
    r = r && fixed_masks_match<3, 0>(dev(3, 0, false));
    r = r && fixed_masks_match<3, 1>(dev(3, 1, false));
    r = r && fixed_masks_match<3, 2>(dev(3, 2, false));
    r = r && fixed_cycles_match<2, 0>(*get_diagram(2, 0));
    // orders 1 and 2: single diagrams and (single-member) groups take the table
    r = r && fixed_labels_match<1, 0>(*get_diagram(1, 0), false) &&
        fixed_labels_match<1, 0>(*get_diagram(1, 0), true);
    r = r && fixed_labels_match<2, 0>(*get_diagram(2, 0), false) &&
        fixed_labels_match<2, 0>(*get_diagram(2, 0), true);
    r = r && fixed_labels_match<3, 0>(*get_diagram(3, 0), false) &&
        fixed_labels_match<3, 1>(*get_diagram(3, 1), false) &&
        fixed_labels_match<3, 2>(*get_diagram(3, 2), false);
    r = r && fixed_cycles_match<3, 0>(*get_diagram(3, 0)) &&
        fixed_cycles_match<3, 1>(*get_diagram(3, 1)) && fixed_cycles_match<3, 2>(*get_diagram(3, 2));
    // the 39 fourth-order diagrams of the per-diagram kernels
    r = r && num_diagrams(4) == 39 &&
        fixed4_match(dev, std::make_integer_sequence<int, 39>{});
    // groups of orders 3 and 4 hold one cycle table per member in LDS
    for (int order = 3; order <= 4; ++order)
      for (int p = 0; p <= order; ++p)
        r = r && group_members(order, p).size() <= static_cast<size_t>(kGroupCycleTables);
    return r;
  }();
  return ok;
}

// Appends one diagram's label tables.  group_base / term_base / coef_base
// are the device element indices at which the three vectors start, so the
// offsets stored in the descriptor are absolute for the kernel's table bases.
bool append_label_tables(const Diagram &d, int q, DiagDev &dd, std::vector<GroupDev> &groups,
                         std::vector<TermDev> &terms, std::vector<double> &coefs,
                         size_t group_base, size_t term_base, size_t coef_base, bool canonical) {
  const LabelTables lt = label_tables(d, q, canonical);
  // label cycles (the nuclear-matter kernels sum over vertex-term choices
  // with them); checked once per diagram against the configuration tables
  const CycleTables ct = cycle_tables(d, canonical);
  if (ct.masks.size() > static_cast<size_t>(kMaxCycles) || ct.of_e.size() > 32) return false;
  dd.ncyc = static_cast<int>(ct.masks.size());
  for (size_t k = 0; k < ct.masks.size(); ++k) dd.cyc_mask[k] = ct.masks[k];
  for (size_t E = 0; E < ct.of_e.size(); ++E) {
    const uint64_t n = static_cast<uint64_t>(ct.n_of_e[E]);
    dd.cyc_e[E] = ct.of_e[E] | n << 56;
    dd.cyc_e32[E] = ct.masks.size() <= 24 ? static_cast<uint32_t>(ct.of_e[E] | n << 24) : 0u;
  }
  {
    static std::mutex mu;
    static std::map<std::tuple<int, int, int, bool>, bool> checked;
    std::lock_guard<std::mutex> lock(mu);
    const auto key = std::make_tuple(d.order, d.id, q, canonical);
    auto it = checked.find(key);
    if (it == checked.end()) it = checked.emplace(key, cycles_match_label_tables(d, q, canonical)).first;
    if (!it->second) return false;
  }
  dd.group_off = static_cast<int>(group_base + groups.size());
  dd.ngroups = static_cast<int>(lt.groups.size());
  dd.term_off = static_cast<int>(term_base + terms.size());
  dd.nterms = static_cast<int>(lt.terms.size());
  const size_t t0 = term_base + terms.size();
  for (const auto &g : lt.groups) {
    GroupDev gd{};
    gd.tau = g.tau;
    gd.first = static_cast<int>(t0 + g.first);
    gd.count = g.count;
    gd.coef_off = static_cast<int>(coef_base + coefs.size());
    const size_t n = g.coef.size(), at = coefs.size();
    coefs.resize(at + coef_slots(d.order), 0.0);
    std::copy(g.coef.begin(), g.coef.end(), coefs.begin() + at);
    float *f = reinterpret_cast<float *>(coefs.data() + at + n);
    for (size_t i = 0; i < n; ++i) f[i] = static_cast<float>(g.coef[i]);
    groups.push_back(gd);
  }
  for (const auto &t : lt.terms) {
    TermDev tm{};
    tm.mult = t.mult;
    tm.codes = t.codes;
    tm.multf = static_cast<float>(t.mult);
    terms.push_back(tm);
  }
  return true;
}

// Medium-dependent task fields: Fermi momenta, loop radii, 1/density, bands.
void fill_medium(const mbpt_context *ctx, double density, double x, TaskDev &T) {
  const double kFn = std::cbrt(3.0 * M_PI * M_PI * ((1.0 - x) * density));
  const double kFp = std::cbrt(3.0 * M_PI * M_PI * (x * density));
  T.kF2[0] = kFn * kFn;
  T.kF2[1] = kFp * kFp;
  const double kFmax = std::max(kFn, kFp);
  T.Rh = kFmax;
  T.Rp = kFmax + ctx->desc.kcut_extra * ctx->v.Lambda;
  T.inv_density = 1.0 / density;
  T.band_k = ctx->desc.fp32_band_k;
  T.band_d = ctx->desc.fp32_band_d;
  T.rel_target = ctx->fp32_rel_target;
  // HF spline range: beyond kF,max + kHfRangeLambda Lambda every partner
  // momentum p exceeds 3 Lambda and the regulator leaves Sigma < 1e-70
  T.hf_h = (kFmax + kHfRangeLambda * ctx->v.Lambda) / kHfIntervals;
  T.hf_inv_h = 1.0 / T.hf_h;
}

// Gauss-Legendre rule on [-1, 1]: the nodes are the zeros of P_n, found by
// Newton's method from cos(pi (i + 3/4) / (n + 1/2)) with P_n and P_n' from
// the three-term recurrence; the weights are 2 / ((1 - x^2) P_n'(x)^2).
void gauss_legendre(int n, double *x, double *w) {
  for (int i = 0; i < n / 2 + n % 2; ++i) {
    double z = std::cos(M_PI * (i + 0.75) / (n + 0.5));
    double d = 0.0;
    for (int it = 0; it < 100; ++it) {
      double p = 1.0, pm = 0.0;
      for (int j = 1; j <= n; ++j) {
        const double pn = ((2 * j - 1) * z * p - (j - 1) * pm) / j;
        pm = p;
        p = pn;
      }
      d = n * (pm - z * p) / (1.0 - z * z);
      const double step = p / d;
      z -= step;
      if (std::fabs(step) <= 1e-16 * std::fabs(z) + 1e-300) {
        // one more evaluation at the converged z for the weight
        p = 1.0;
        pm = 0.0;
        for (int j = 1; j <= n; ++j) {
          const double pn = ((2 * j - 1) * z * p - (j - 1) * pm) / j;
          pm = p;
          p = pn;
        }
        d = n * (pm - z * p) / (1.0 - z * z);
        break;
      }
    }
    x[n - 1 - i] = z;
    x[i] = -z;
    w[i] = w[n - 1 - i] = 2.0 / ((1.0 - z * z) * d * d);
  }
}

// Compile a task list's diagrams into device tables (one descriptor per
// distinct (order, id)).
int compile_task_diagrams(mbpt_context *ctx, int q, int order, int id, bool group,
                          std::vector<DiagDev> &dds, std::vector<GroupDev> &groups,
                          std::vector<TermDev> &terms, std::vector<double> &coefs,
                          FlopModel &model) {
  const std::vector<int> ids = group ? group_members(order, id) : std::vector<int>{id};
  if (ids.empty()) {
    set_err(ctx, "unknown diagram or empty diagram group");
    return MBPT_EINVAL;
  }
  model = FlopModel{};
  double units = 0.0, unit_flops = 0.0;
  for (size_t i = 0; i < ids.size(); ++i) {
    const Diagram *d = get_diagram(order, ids[i]);
    if (!d) {
      set_err(ctx, "unknown diagram");
      return MBPT_EINVAL;
    }
    DiagDev dd{};
    dd.order = d->order;
    dd.id = d->id;
    dd.nlines = d->nlines;
    dd.nloops = d->nloops;
    dd.ncuts = d->ncuts;
    fill_diag_dev(*d, dd, group);
    if (!append_label_tables(*d, q, dd, groups, terms, coefs, 0, 0, 0, group)) {
      set_err(ctx, "label cycle tables disagree with the label tables");
      return MBPT_EINVAL;
    }
    dds.push_back(dd);
    FlopModel fm;
    count_flops(*d, q, ctx->v.reg_exp / 2, ctx->desc.label_mode, ctx->desc.spectrum, fm);
    // the nuclear-matter factorised label sum of a single diagram with the
    // free spectrum is the cycle form: one polynomial per passing sample
    fm.all_units = ctx->desc.label_mode ? dd.nterms
                   : (q == 4 && !group && ctx->desc.spectrum == MBPT_SPECTRUM_FREE)
                       ? 1
                       : dd.ngroups;
    // a group shares the map and loop momenta; its pass and label-unit
    // counters add up over members, so post and per_term are averages
    model.pre += i == 0 ? fm.pre : fm.pre - fm.shared;
    model.shared = fm.shared;
    model.post += fm.post / ids.size();
    model.transc_pre += i == 0 ? fm.transc_pre : fm.transc_pre - fm.transc_shared;
    model.transc_shared = fm.transc_shared;
    model.transc_post += fm.transc_post / ids.size();
    units += fm.all_units;
    unit_flops += fm.per_term * fm.all_units;
  }
  model.all_units = units;
  model.per_term = units > 0.0 ? unit_flops / units : 0.0;
  return MBPT_OK;
}

int compile_tables(mbpt_task_set *set) {
  mbpt_context *ctx = set->ctx;
  const int q = set->q;
  set->diags.clear();
  set->groups.clear();
  set->terms.clear();
  set->coefs.clear();
  set->task_diag.assign(set->tasks.size(), -1);
  set->task_ndiag.assign(set->tasks.size(), 1);
  set->flops.assign(set->tasks.size(), FlopModel{});
  // one entry per distinct (order, id, group): first descriptor, count, model
  struct Entry {
    int order, id, group, first, count;
    FlopModel fm;
  };
  std::vector<Entry> done;
  for (size_t t = 0; t < set->tasks.size(); ++t) {
    const auto &td = set->tasks[t];
    const Entry *hit = nullptr;
    for (const auto &e : done)
      if (e.order == td.order && e.id == td.diagram_id && e.group == td.group) hit = &e;
    if (!hit) {
      Entry e{td.order, td.diagram_id, td.group, static_cast<int>(set->diags.size()), 0,
              FlopModel{}};
      const int rc = compile_task_diagrams(ctx, q, td.order, td.diagram_id, td.group != 0,
                                           set->diags, set->groups, set->terms, set->coefs, e.fm);
      if (rc) return rc;
      e.count = static_cast<int>(set->diags.size()) - e.first;
      done.push_back(e);
      hit = &done.back();
    }
    set->task_diag[t] = hit->first;
    set->task_ndiag[t] = hit->count;
    set->flops[t] = hit->fm;
  }
  set->max_nd = 0;
  for (const auto &td : set->tasks) set->max_nd = std::max(set->max_nd, 3 * (td.order + 1));
  return MBPT_OK;
}

// Host copy of the per-task parameters (the state part is device-owned).
void fill_task_params(mbpt_task_set *set) {
  mbpt_context *ctx = set->ctx;
  const int nb = ctx->desc.n_bins;
  set->h_tasks.assign(set->tasks.size(), TaskDev{});
  int goff = 0, hoff = 0;
  for (size_t t = 0; t < set->tasks.size(); ++t) {
    const auto &td = set->tasks[t];
    TaskDev &T = set->h_tasks[t];
    const int nd = 3 * (td.order + 1);
    T.diag = set->task_diag[t];
    T.ndiag = set->task_ndiag[t];
    T.nd = nd;
    T.hf_off = static_cast<int>(t) * 2 * kHfEntries;
    T.grid_off = goff;
    T.hist_off = hoff;
    goff += nd * (nb + 1);
    hoff += nd * nb;
    T.res_off = static_cast<int>(t) * set->max_iters;
    T.res_cap = set->max_iters;
    T.key = td.task_key;
    T.order = td.order;
    fill_medium(ctx, td.density, td.proton_fraction, T);
    T.active = 1;
    T.plan = 0x7fffffff;  // every iteration
    T.train_iters = set->train_iters;
  }
  set->grid_doubles = goff;
  set->hist_doubles = hoff;
}

size_t items_for(const mbpt_task_set *set, uint64_t samples) {
  const uint64_t chunk = static_cast<uint64_t>(set->block) * set->spt;
  return static_cast<size_t>((samples + chunk - 1) / chunk);
}

// Samples per thread unless set explicitly, chosen at bind for the launch
// mode the set has then: the larger of (a) a task's max_samples spread over
// about two blocks per CU, at most 16 (one task's iteration lasts as long as
// its slowest block), and (b) the samples of one launch spread over about 16
// blocks per CU, at most 256 (a launch covers one task in the per-task mode,
// all the tasks of an order otherwise): large work items halve the per-item
// costs (grid and tables into LDS, the histogram merge, the last partial
// fp64 re-evaluation round of the fp32 path) while a launch still spans many
// rounds of blocks.
int auto_spt(const mbpt_task_set *set, uint64_t max_samples) {
  const uint64_t cus = static_cast<uint64_t>(std::max(1, set->ctx->num_cus));
  const uint64_t a =
      std::max<uint64_t>(1, std::min<uint64_t>(16, max_samples / (set->block * 2 * cus)));
  uint64_t per_launch = max_samples;
  if (set->launch_mode != MBPT_LAUNCH_PER_TASK) {
    int count[kMaxOrder + 1] = {};
    int most = 1;
    for (const auto &t : set->tasks)
      if (t.order >= 1 && t.order <= kMaxOrder) most = std::max(most, ++count[t.order]);
    per_launch = max_samples * static_cast<uint64_t>(most);
  }
  const uint64_t b = std::min<uint64_t>(256, per_launch / (set->block * 16 * cus));
  return static_cast<int>(std::max(a, b));
}

struct Layout {
  size_t tasks, olist, diags, groups, terms, coefs, grids, hists, partials, counters, reslog, hf,
      gl, cpart, creslog, queue, total;
};

Layout layout_of(const mbpt_task_set *set, uint64_t max_samples, int max_iters, int nb) {
  // item capacity for the blocking the set will have once bound
  const uint64_t chunk = static_cast<uint64_t>(set->block) *
                         (set->blocking_auto ? auto_spt(set, max_samples) : set->spt);
  const size_t items_per_task = static_cast<size_t>((max_samples + chunk - 1) / chunk);
  Layout L{};
  size_t off = 0;
  const size_t nt = set->tasks.size();
  L.tasks = off;
  off = align256(off + nt * sizeof(TaskDev));
  L.olist = off;
  off = align256(off + nt * sizeof(int2));
  L.diags = off;
  off = align256(off + set->diags.size() * sizeof(DiagDev));
  L.groups = off;
  off = align256(off + std::max<size_t>(1, set->groups.size()) * sizeof(GroupDev));
  L.terms = off;
  off = align256(off + std::max<size_t>(1, set->terms.size()) * sizeof(TermDev));
  L.coefs = off;
  off = align256(off + std::max<size_t>(1, set->coefs.size()) * sizeof(double));
  size_t gd = 0, hd = 0;
  for (const auto &td : set->tasks) {
    gd += 3 * (td.order + 1) * (nb + 1);
    hd += 3 * (td.order + 1) * nb;
  }
  L.grids = off;
  off = align256(off + gd * sizeof(double));
  L.hists = off;
  off = align256(off + hd * sizeof(double));
  const size_t items = nt * items_per_task;
  L.partials = off;
  off = align256(off + items * 4 * sizeof(double));
  L.counters = off;
  off = align256(off + items * kItemCounters * sizeof(uint64_t));
  L.reslog = off;
  off = align256(off + nt * static_cast<size_t>(std::max(1, max_iters)) * 2 * sizeof(double));
  L.hf = off;  // two isospin tables per task, used with the HF spectrum
  off = align256(off + nt * 2 * static_cast<size_t>(kHfEntries) * 4 * sizeof(double));
  L.gl = off;
  off = align256(off + 2 * kHfGauss * sizeof(double));
  // regularised components: per-item sums and per-iteration estimates
  L.cpart = off;
  off = align256(off + items * kRegSums * sizeof(double));
  L.creslog = off;
  off = align256(off + nt * static_cast<size_t>(std::max(1, max_iters)) * kRegSums *
                           sizeof(double));
  L.queue = off;  // work-item counters of the persistent launches
  off = align256(off + kQueueSlots * sizeof(int));
  L.total = off;
  return L;
}

KArgs kargs_of(const mbpt_task_set *set) {
  const mbpt_context *ctx = set->ctx;
  KArgs a{};
  a.tasks = set->d_tasks;
  a.diags = set->d_diags;
  a.groups = set->d_groups;
  a.terms = set->d_terms;
  a.gcoef = set->d_coefs;
  a.olist = set->d_olist;
  a.hf = set->d_hf;
  a.grids = set->d_grids;
  a.hists = set->d_hists;
  a.partials = set->d_partials;
  a.counters = set->d_counters;
  a.reslog = set->d_reslog;
  a.cpart = set->d_cpart;
  a.creslog = set->d_creslog;
  a.queue = set->d_queue;
  a.nreg = ctx->reg_n;
  a.reg_eta = ctx->reg_eta;
  extrapolation_weights(ctx->reg_n, a.reg_coef);
  a.ntasks = static_cast<int>(set->tasks.size());
  a.total_items = 0;
  a.spt = set->spt;
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
  a.phys.spectrum = ctx->desc.spectrum;
  return a;
}

// Precision, interaction or spectrum changed since the set last ran: captured
// launches, launch shapes and HF tables are stale.
int upload_params(mbpt_task_set *set);

int sync_epoch(mbpt_task_set *set) {
  if (set->epoch == set->ctx->epoch) return MBPT_OK;
  set->drop_graph();
  set->oranges.clear();
  set->hf_dirty = true;
  // context settings the tasks carry (uploaded with the parameters)
  for (auto &T : set->h_tasks) {
    T.band_k = set->ctx->desc.fp32_band_k;
    T.band_d = set->ctx->desc.fp32_band_d;
    T.rel_target = set->ctx->fp32_rel_target;
  }
  set->epoch = set->ctx->epoch;
  return set->ws ? upload_params(set) : MBPT_OK;
}

// (Re)computes the HF spline tables of every task when the spectrum is HF and
// the medium, interaction or spectrum changed since they were made.
int ensure_hf(mbpt_task_set *set) {
  mbpt_context *ctx = set->ctx;
  if (!ctx->desc.spectrum || !set->hf_dirty) return MBPT_OK;
  const KArgs a = kargs_of(set);
  HIPCHK(ctx, launch_hf(a, set->d_gl, 0, static_cast<int>(set->tasks.size()),
                        set->q == 4 ? 2 : 1, set->q == 4 ? 2 : 1, ctx->stream));
  set->hf_dirty = false;
  return MBPT_OK;
}

// Upload the parameter prefix of every TaskDev (state left untouched).
int upload_params(mbpt_task_set *set) {
  mbpt_context *ctx = set->ctx;
  const size_t width = offsetof(TaskDev, iter);
  HIPCHK(ctx, hipMemcpy2DAsync(set->d_tasks, sizeof(TaskDev), set->h_tasks.data(), sizeof(TaskDev),
                               width, set->h_tasks.size(), hipMemcpyHostToDevice, ctx->stream));
  if (!set->olist.empty())
    HIPCHK(ctx, hipMemcpyAsync(set->d_olist, set->olist.data(), set->olist.size() * sizeof(int2),
                               hipMemcpyHostToDevice, ctx->stream));
  return MBPT_OK;
}

int bind(mbpt_task_set *set, void *ptr, size_t bytes, uint64_t max_samples, int max_iters) {
  mbpt_context *ctx = set->ctx;
  const int nb = ctx->desc.n_bins;
  if (!ptr || (reinterpret_cast<uintptr_t>(ptr) & 255u) || max_samples < 2 || max_iters < 1) {
    set_err(ctx, "bind_workspace: null or misaligned pointer, or bad limits");
    return MBPT_EINVAL;
  }
  const Layout L = layout_of(set, max_samples, max_iters, nb);
  if (bytes < L.total) {
    set_err(ctx, "bind_workspace: workspace too small (" + std::to_string(bytes) + " < " +
                     std::to_string(L.total) + ")");
    return MBPT_ENOMEM;
  }
  char *base = static_cast<char *>(ptr);
  set->ws = base;
  set->ws_bytes = bytes;
  set->max_samples = max_samples;
  set->max_iters = max_iters;
  if (set->blocking_auto) set->spt = auto_spt(set, max_samples);
  set->max_items = set->tasks.size() * items_for(set, max_samples);
  set->d_tasks = reinterpret_cast<TaskDev *>(base + L.tasks);
  set->d_olist = reinterpret_cast<int2 *>(base + L.olist);
  set->d_diags = reinterpret_cast<DiagDev *>(base + L.diags);
  set->d_groups = reinterpret_cast<GroupDev *>(base + L.groups);
  set->d_terms = reinterpret_cast<TermDev *>(base + L.terms);
  set->d_coefs = reinterpret_cast<double *>(base + L.coefs);
  set->d_grids = reinterpret_cast<double *>(base + L.grids);
  set->d_hists = reinterpret_cast<double *>(base + L.hists);
  set->d_partials = reinterpret_cast<double *>(base + L.partials);
  set->d_counters = reinterpret_cast<uint64_t *>(base + L.counters);
  set->d_reslog = reinterpret_cast<double *>(base + L.reslog);
  set->d_hf = reinterpret_cast<double *>(base + L.hf);
  set->d_gl = reinterpret_cast<double *>(base + L.gl);
  set->d_cpart = reinterpret_cast<double *>(base + L.cpart);
  set->d_creslog = reinterpret_cast<double *>(base + L.creslog);
  set->d_queue = reinterpret_cast<int *>(base + L.queue);
  set->run_reg_n = -1;
  set->h_gl.assign(2 * kHfGauss, 0.0);
  gauss_legendre(kHfGauss, set->h_gl.data(), set->h_gl.data() + kHfGauss);
  HIPCHK(ctx, hipMemcpyAsync(set->d_gl, set->h_gl.data(), set->h_gl.size() * sizeof(double),
                             hipMemcpyHostToDevice, ctx->stream));
  set->hf_dirty = true;
  fill_task_params(set);
  set->oranges.clear();
  HIPCHK(ctx, hipMemcpyAsync(set->d_diags, set->diags.data(), set->diags.size() * sizeof(DiagDev),
                             hipMemcpyHostToDevice, ctx->stream));
  if (!set->groups.empty())
    HIPCHK(ctx, hipMemcpyAsync(set->d_groups, set->groups.data(),
                               set->groups.size() * sizeof(GroupDev), hipMemcpyHostToDevice,
                               ctx->stream));
  if (!set->terms.empty())
    HIPCHK(ctx, hipMemcpyAsync(set->d_terms, set->terms.data(), set->terms.size() * sizeof(TermDev),
                               hipMemcpyHostToDevice, ctx->stream));
  if (!set->coefs.empty())
    HIPCHK(ctx, hipMemcpyAsync(set->d_coefs, set->coefs.data(), set->coefs.size() * sizeof(double),
                               hipMemcpyHostToDevice, ctx->stream));
  int rc = upload_params(set);
  if (rc) return rc;
  KArgs a = kargs_of(set);
  HIPCHK(ctx, launch_init(a, 0, static_cast<int>(set->tasks.size()), ctx->stream));
  HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
  set->drop_graph();
  set->last_state.clear();
  return MBPT_OK;
}

static hipEvent_t new_event() {
  hipEvent_t e = nullptr;
  (void)hipEventCreate(&e);
  return e;
}

// Timing events around sample launches, resolved after the stream drains.
void timed_begin(mbpt_context *ctx, size_t &slot) {
  if (ctx->n_used == ctx->events.size()) ctx->events.emplace_back(new_event(), new_event());
  slot = ctx->n_used++;
  (void)hipEventRecord(ctx->events[slot].first, ctx->stream);
}

void timed_end(mbpt_context *ctx, size_t slot) { (void)hipEventRecord(ctx->events[slot].second, ctx->stream); }

void resolve_timing(mbpt_context *ctx) {
  for (size_t i = 0; i < ctx->n_used; ++i) {
    float ms = 0.0f;
    if (hipEventElapsedTime(&ms, ctx->events[i].first, ctx->events[i].second) == hipSuccess)
      ctx->kernel_ms += ms;
    ctx->launches += 1;
  }
  ctx->n_used = 0;
}

void result_of(const TaskDev &S, mbpt_result &r) {
  r = mbpt_result{};
  r.iters_done = S.it_done;
  r.n_evals = S.nevals;
  r.n_fp64_fallback = S.nfallback;
  r.last_E = S.lastI;
  r.last_sigma = std::sqrt(std::max(0.0, S.lastV));
  if (S.it_done == 0) return;
  if (S.nzero > 0) {
    r.E_per_A = S.zsum / S.nzero;
    r.sigma = 0.0;
    r.chi2_dof = 0.0;
  } else {
    r.E_per_A = S.wisum / S.wsum;
    r.sigma = 1.0 / std::sqrt(S.wsum);
    const double chi2 = S.wi2sum - S.wisum * S.wisum / S.wsum;
    r.chi2_dof = S.ncomb > 1 ? std::max(0.0, chi2) / (S.ncomb - 1) : 0.0;
  }
}

}  // namespace mbpt

static int check_tasks(mbpt_context *ctx, const mbpt_task_desc *tasks, int n, int *q) {
  if (!tasks || n < 1) return MBPT_EINVAL;
  int matter = tasks[0].matter;
  for (int i = 0; i < n; ++i) {
    const auto &t = tasks[i];
    if (t.matter != matter || (t.matter != MBPT_NEUTRON && t.matter != MBPT_NUCLEAR)) {
      set_err(ctx, "task set: every task needs the same matter (NEUTRON or NUCLEAR)");
      return MBPT_EINVAL;
    }
    if (t.group != 0 && t.group != 1) {
      set_err(ctx, "task set: group must be 0 (one diagram) or 1 (a diagram group)");
      return MBPT_EINVAL;
    }
    if (t.group ? group_members(t.order, t.diagram_id).empty() : !get_diagram(t.order, t.diagram_id)) {
      set_err(ctx, "task set: unknown diagram or empty diagram group");
      return MBPT_EINVAL;
    }
    if (t.group && ctx->desc.spectrum != MBPT_SPECTRUM_FREE) {
      set_err(ctx, "task set: diagram groups take the free spectrum only");
      return MBPT_EINVAL;
    }
    if (!(t.density > 0.0) || !(t.proton_fraction >= 0.0 && t.proton_fraction <= 1.0) ||
        (t.matter == MBPT_NEUTRON && t.proton_fraction != 0.0)) {
      set_err(ctx, "task set: density must be > 0, proton fraction in [0,1] (0 for NEUTRON)");
      return MBPT_EINVAL;
    }
  }
  *q = matter == MBPT_NUCLEAR ? 4 : 2;
  return MBPT_OK;
}

extern "C" int mbpt_create_task_set(mbpt_context *ctx, const mbpt_task_desc *tasks, int n_tasks,
                                    mbpt_task_set **out) {
  if (!ctx || !out) return MBPT_EINVAL;
  *out = nullptr;
  if (!fixed_masks_ok()) {
    set_err(ctx, "internal: the generator's descriptors differ from the kernels' compile-time "
                 "tables or exceed their group limit");
    return MBPT_EINVAL;
  }
  int q = 2;
  int rc = check_tasks(ctx, tasks, n_tasks, &q);
  if (rc) return rc;
  auto *set = new mbpt_task_set();
  set->ctx = ctx;
  set->q = q;
  set->tasks.assign(tasks, tasks + n_tasks);
  rc = compile_tables(set);
  if (rc) {
    delete set;
    return rc;
  }
  *out = set;
  return MBPT_OK;
}

extern "C" int mbpt_create_diagram_set_from_order(mbpt_context *ctx, int order, const int *ids,
                                                  int n_ids, int matter, mbpt_task_set **out) {
  if (!ctx || !out) return MBPT_EINVAL;
  const int nd = num_diagrams(order);
  if (nd < 0) return MBPT_EINVAL;
  std::vector<mbpt_task_desc> ts;
  const int n = ids ? n_ids : nd;
  for (int i = 0; i < n; ++i) {
    mbpt_task_desc t{};
    t.order = order;
    t.diagram_id = ids ? ids[i] : i;
    t.matter = matter;
    t.density = 0.16;
    t.proton_fraction = 0.0;
    t.task_key = static_cast<uint32_t>(i);
    ts.push_back(t);
  }
  if (ts.empty()) return MBPT_EINVAL;
  return mbpt_create_task_set(ctx, ts.data(), static_cast<int>(ts.size()), out);
}

extern "C" int mbpt_diagram_desc_id(const mbpt_diagram_desc *d, int *id) {
  if (!d || !id) return MBPT_EINVAL;
  std::string err;
  const int r = diagram_from_lines(d->order, d->nlines, d->line_from, d->line_to, d->vertex, err);
  if (r < 0) return MBPT_EINVAL;
  *id = r;
  return MBPT_OK;
}

extern "C" int mbpt_diagram_desc_of(int order, int id, mbpt_diagram_desc *out) {
  const Diagram *d = get_diagram(order, id);
  if (!d || !out) return MBPT_EINVAL;
  *out = mbpt_diagram_desc{};
  out->order = d->order;
  out->nlines = d->nlines;
  for (int l = 0; l < d->nlines; ++l) {
    out->line_from[l] = d->tail[l];
    out->line_to[l] = d->head[l];
  }
  for (int v = 0; v < d->order; ++v) {
    out->vertex[v][0] = d->vout[v][0];
    out->vertex[v][1] = d->vout[v][1];
    out->vertex[v][2] = d->vin[v][0];
    out->vertex[v][3] = d->vin[v][1];
  }
  return MBPT_OK;
}

extern "C" int mbpt_create_diagram_set(mbpt_context *ctx, const mbpt_diagram_desc *descs, int n,
                                       int matter, mbpt_task_set **out) {
  if (!ctx || !out || !descs || n < 1) return MBPT_EINVAL;
  *out = nullptr;
  std::vector<mbpt_task_desc> ts;
  for (int i = 0; i < n; ++i) {
    std::string err;
    const mbpt_diagram_desc &d = descs[i];
    const int id = diagram_from_lines(d.order, d.nlines, d.line_from, d.line_to, d.vertex, err);
    if (id < 0) {
      set_err(ctx, "create_diagram_set: descriptor " + std::to_string(i) + ": " + err);
      return MBPT_EINVAL;
    }
    mbpt_task_desc t{};
    t.order = d.order;
    t.diagram_id = id;
    t.matter = matter;
    t.density = 0.16;
    t.proton_fraction = 0.0;
    t.task_key = static_cast<uint32_t>(i);
    ts.push_back(t);
  }
  return mbpt_create_task_set(ctx, ts.data(), n, out);
}

extern "C" void mbpt_task_set_destroy(mbpt_task_set *set) {
  if (!set) return;
  set->drop_graph();
  delete set;
}

extern "C" int mbpt_task_count(const mbpt_task_set *set, int *n) {
  if (!set || !n) return MBPT_EINVAL;
  *n = static_cast<int>(set->tasks.size());
  return MBPT_OK;
}

namespace mbpt {
// A task set moved to another EOS point: new medium parameters, running sums,
// counters and iteration logs restarted (the old point's iterations estimate
// another integral), grids and Philox iteration words kept (warm start).
static int move_eos_point(mbpt_task_set *set) {
  set->drop_graph();
  set->hf_dirty = true;
  if (!set->ws) return MBPT_OK;
  fill_task_params(set);
  int rc = upload_params(set);
  if (rc) return rc;
  mbpt_context *ctx = set->ctx;
  KArgs a = kargs_of(set);
  HIPCHK(ctx, launch_init(a, 0, static_cast<int>(set->tasks.size()), ctx->stream, true));
  HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
  set->last_state.clear();
  set->run_reg_n = -1;
  return MBPT_OK;
}
}  // namespace mbpt

extern "C" int mbpt_set_density(mbpt_task_set *set, double density) {
  if (!set || !(density > 0.0)) return MBPT_EINVAL;
  for (auto &t : set->tasks) t.density = density;
  return move_eos_point(set);
}

extern "C" int mbpt_set_asymmetry(mbpt_task_set *set, double x) {
  if (!set || !(x >= 0.0 && x <= 1.0)) return MBPT_EINVAL;
  if (set->q == 2 && x != 0.0) {
    set_err(set->ctx, "set_asymmetry: neutron matter needs proton fraction 0");
    return MBPT_EINVAL;
  }
  for (auto &t : set->tasks) t.proton_fraction = x;
  return move_eos_point(set);
}

extern "C" int mbpt_set_training(mbpt_task_set *set, int train_iters) {
  if (!set || train_iters < 0) return MBPT_EINVAL;
  set->train_iters = train_iters;
  for (auto &T : set->h_tasks) T.train_iters = train_iters;
  set->drop_graph();
  if (!set->ws) return MBPT_OK;
  return upload_params(set);
}

extern "C" int mbpt_set_launch_mode(mbpt_task_set *set, int mode) {
  if (!set || mode < MBPT_LAUNCH_PER_TASK || mode > MBPT_LAUNCH_PERSISTENT) return MBPT_EINVAL;
  set->launch_mode = mode;
  set->drop_graph();
  set->oranges.clear();
  return MBPT_OK;
}

extern "C" int mbpt_get_blocking(const mbpt_task_set *set, int *threads_per_block,
                                 int *samples_per_thread) {
  if (!set || !threads_per_block || !samples_per_thread) return MBPT_EINVAL;
  *threads_per_block = set->block;
  *samples_per_thread = set->spt;
  return MBPT_OK;
}

extern "C" int mbpt_set_blocking(mbpt_task_set *set, int threads_per_block, int samples_per_thread) {
  if (!set || threads_per_block < 64 || threads_per_block > 256 || (threads_per_block % 64) ||
      samples_per_thread < 1 || samples_per_thread > 256)
    return MBPT_EINVAL;
  if (set->ws && static_cast<size_t>(threads_per_block) * samples_per_thread <
                     static_cast<size_t>(set->block) * set->spt) {
    set_err(set->ctx, "set_blocking: smaller work items than at bind time need a larger workspace");
    return MBPT_ESTATE;
  }
  set->block = threads_per_block;
  set->spt = samples_per_thread;
  set->blocking_auto = false;
  set->drop_graph();
  set->oranges.clear();
  return MBPT_OK;
}

extern "C" int mbpt_workspace_query(const mbpt_task_set *set, uint64_t max_samples_per_iter,
                                    int max_iters, size_t *bytes) {
  if (!set || !bytes || max_samples_per_iter < 2 || max_iters < 1) return MBPT_EINVAL;
  *bytes = layout_of(set, max_samples_per_iter, max_iters, set->ctx->desc.n_bins).total;
  return MBPT_OK;
}

extern "C" int mbpt_bind_workspace(mbpt_task_set *set, void *device_ptr, size_t bytes,
                                   uint64_t max_samples_per_iter, int max_iters) {
  if (!set) return MBPT_EINVAL;
  return bind(set, device_ptr, bytes, max_samples_per_iter, max_iters);
}

extern "C" int mbpt_reset(mbpt_task_set *set) {
  if (!set) return MBPT_EINVAL;
  if (!set->ws) return MBPT_ESTATE;
  mbpt_context *ctx = set->ctx;
  KArgs a = kargs_of(set);
  HIPCHK(ctx, launch_init(a, 0, static_cast<int>(set->tasks.size()), ctx->stream));
  HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
  set->last_state.clear();
  set->run_reg_n = -1;
  return MBPT_OK;
}

namespace mbpt {

// Queue `iters` iterations of the whole set on the context stream.
int enqueue_iterations(mbpt_task_set *set, KArgs &a, int iters, bool timed) {
  mbpt_context *ctx = set->ctx;
  const int nt = static_cast<int>(set->tasks.size());
  const double alpha = ctx->desc.alpha;
  if (set->launch_mode == MBPT_LAUNCH_PER_TASK) {
    // one sample launch per task and iteration; the iteration ends of all
    // tasks (independent of each other) share one launch
    for (int it = 0; it < iters; ++it) {
      for (int t = 0; t < nt; ++t) {
        size_t slot = 0;
        if (timed) timed_begin(ctx, slot);
        HIPCHK(ctx, launch_sample_single(a, t, set->tasks[t].order, set->q, ctx->desc.precision,
                                         set->task_ndiag[t] > 1,
                                         set->h_tasks[t].nitems, set->block, ctx->stream));
        if (timed) timed_end(ctx, slot);
      }
      HIPCHK(ctx, launch_finish(a, 0, nt, 0, alpha, ctx->stream));
    }
    return MBPT_OK;
  }
  const bool persistent = set->launch_mode == MBPT_LAUNCH_PERSISTENT;
  // fourth-order nuclear-matter single diagrams with the quartic regulator,
  // the polynomial label sums and the free spectrum take the per-diagram
  // kernels (compile-time masks): one launch per diagram of the order's range
  // (the tasks are numbered by diagram, see mbpt_integrate)
  const int prec = ctx->desc.precision;
  auto fixed4 = [&](const OrderRange &r) {
    return !persistent && r.order == 4 && set->q == 4 && !r.group && ctx->desc.label_mode == 0 &&
           a.phys.half_exp == 2 && a.phys.spectrum == MBPT_SPECTRUM_FREE && a.nreg == 0 &&
           (prec == MBPT_FP64 || prec == MBPT_FP32);
  };
  auto id_of = [&](int k) { return set->diags[set->task_diag[set->olist[k].y]].id; };
  for (int it = 0; it < iters; ++it) {
    size_t slot = 0;
    if (timed) timed_begin(ctx, slot);
    for (const auto &r : set->oranges) {
      if (persistent) {
        HIPCHK(ctx, launch_sample_persistent(a, r.order, set->q, prec, r.group, r.k0, r.k1,
                                             r.nitems, set->block, ctx->num_cus, ctx->stream));
      } else if (fixed4(r)) {
        for (int ka = r.k0; ka < r.k1;) {
          const int id = id_of(ka);
          int kb = ka + 1;
          while (kb < r.k1 && id_of(kb) == id) ++kb;
          const int end = kb < r.k1 ? set->olist[kb].x : r.item_end;
          HIPCHK(ctx, launch_sample_order_fixed4(a, id, prec == MBPT_FP32 ? 1 : 0, ka, kb,
                                                 end - set->olist[ka].x, set->block, ctx->stream));
          ka = kb;
        }
      } else {
        HIPCHK(ctx, launch_sample_order(a, r.order, set->q, prec, r.group, r.k0, r.k1, r.nitems,
                                        set->block, ctx->stream));
      }
    }
    if (timed) timed_end(ctx, slot);
    HIPCHK(ctx, launch_finish(a, 0, nt, 0, alpha, ctx->stream));
  }
  return MBPT_OK;
}

// Work numbering grouped by order: the tasks of each order own a contiguous
// item range, listed in olist as (first item, task), so one launch per order
// (one block per item) covers them.
void order_items(std::vector<TaskDev> &T, const std::vector<int> &active,
                 std::vector<int2> &olist, std::vector<OrderRange> &ranges) {
  olist.clear();
  ranges.clear();
  int item = 0;
  for (int o = 1; o <= kMaxOrder; ++o) {
    const int k0 = static_cast<int>(olist.size());
    for (int t : active) {
      if (T[t].order != o) continue;
      T[t].item_begin = item;
      olist.push_back(make_int2(item, t));
      item += T[t].nitems;
    }
    const int k1 = static_cast<int>(olist.size());
    if (k1 == k0) continue;
    OrderRange r{};
    r.order = o;
    r.k0 = k0;
    r.k1 = k1;
    r.item_end = item;
    r.nitems = item - olist[k0].x;
    r.group = false;
    for (int k = k0; k < k1; ++k) r.group = r.group || T[olist[k].y].ndiag > 1;
    ranges.push_back(r);
  }
}

}  // namespace mbpt

extern "C" int mbpt_integrate(mbpt_task_set *set, uint64_t samples_per_iter, int iters,
                              mbpt_result *per_task, mbpt_result *total) {
  if (!set || iters < 1 || samples_per_iter < 2) return MBPT_EINVAL;
  mbpt_context *ctx = set->ctx;
  if (!set->ws) {
    set_err(ctx, "integrate: no workspace bound");
    return MBPT_ESTATE;
  }
  if (samples_per_iter > set->max_samples) {
    set_err(ctx, "integrate: samples_per_iter exceeds the bound limit");
    return MBPT_ENOMEM;
  }
  const int nt = static_cast<int>(set->tasks.size());
  // work items
  int item = 0;
  const int per = static_cast<int>(items_for(set, samples_per_iter));
  if (static_cast<size_t>(per) * nt > set->max_items) {
    set_err(ctx, "integrate: more work items than the workspace holds");
    return MBPT_ENOMEM;
  }
  // the component log holds one regularisation per run from a reset
  if (ctx->reg_n > 0 && ctx->desc.spectrum != MBPT_SPECTRUM_FREE) {
    set_err(ctx, "integrate: regularised components take the free spectrum only");
    return MBPT_ESTATE;
  }
  if (set->run_reg_n >= 0 &&
      (set->run_reg_n != ctx->reg_n || set->run_reg_eta != ctx->reg_eta)) {
    set_err(ctx, "integrate: regularisation changed since the set's iterations began (reset first)");
    return MBPT_ESTATE;
  }
  set->run_reg_n = ctx->reg_n;
  set->run_reg_eta = ctx->reg_eta;
  {
    const int rc = sync_epoch(set);
    if (rc) return rc;
  }
  bool changed = false;
  std::vector<int> all(nt);
  for (int t = 0; t < nt; ++t) {
    TaskDev &T = set->h_tasks[t];
    all[t] = t;
    changed |= T.nitems != per || T.nsamples != samples_per_iter;
    T.nitems = per;
    T.nsamples = samples_per_iter;
  }
  // within an order, tasks numbered by diagram (the per-diagram kernels take
  // one diagram's tasks per launch)
  std::stable_sort(all.begin(), all.end(), [&](int x, int y) {
    return set->diags[set->task_diag[x]].id < set->diags[set->task_diag[y]].id;
  });
  if (changed || set->oranges.empty()) {
    order_items(set->h_tasks, all, set->olist, set->oranges);
    for (int t = 0; t < nt; ++t) set->h_tasks[t].store_begin = set->h_tasks[t].item_begin;
    item = set->oranges.back().item_end;
    changed = true;
  } else {
    item = set->oranges.back().item_end;
  }
  if (changed) {
    set->drop_graph();
    int rc = upload_params(set);
    if (rc) return rc;
  }
  {
    const int rc = ensure_hf(set);
    if (rc) return rc;
  }
  KArgs a = kargs_of(set);
  a.total_items = item;
  uint64_t evals_before = 0;
  {
    int rc = 0;
    if (set->launch_mode == MBPT_LAUNCH_GRAPH && !set->noalloc) {
      if (ctx->stream == nullptr) {
        set_err(ctx, "integrate: GRAPH launch mode needs a non-default stream to capture on");
        return MBPT_EINVAL;
      }
      if (!set->graph_exec || set->graph_iters != iters) {
        set->drop_graph();
        hipGraph_t graph = nullptr;
        HIPCHK(ctx, hipStreamBeginCapture(ctx->stream, hipStreamCaptureModeThreadLocal));
        rc = enqueue_iterations(set, a, iters, false);
        hipError_t e = hipStreamEndCapture(ctx->stream, &graph);
        if (rc) return rc;
        if (e != hipSuccess) return hip_fail(ctx, e, "hipStreamEndCapture");
        e = hipGraphInstantiate(&set->graph_exec, graph, nullptr, nullptr, 0);
        (void)hipGraphDestroy(graph);
        if (e != hipSuccess) return hip_fail(ctx, e, "hipGraphInstantiate");
        set->graph_iters = iters;
      }
      size_t slot = 0;
      timed_begin(ctx, slot);
      HIPCHK(ctx, hipGraphLaunch(set->graph_exec, ctx->stream));
      timed_end(ctx, slot);
    } else {
      rc = enqueue_iterations(set, a, iters, !set->noalloc);
      if (rc) return rc;
    }
  }
  (void)evals_before;
  std::vector<TaskDev> st(nt);
  HIPCHK(ctx, hipMemcpyAsync(st.data(), set->d_tasks, nt * sizeof(TaskDev), hipMemcpyDeviceToHost,
                             ctx->stream));
  HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
  resolve_timing(ctx);
  // FLOP accounting from the device counters of this call
  uint64_t evals = 0;
  double flops = 0.0;
  for (int t = 0; t < nt; ++t) {
    const TaskDev &S = st[t];
    const TaskDev &P = set->last_state.empty() ? TaskDev{} : set->last_state[t];
    const uint64_t de = S.nevals - P.nevals, dp = S.npass - P.npass, dt = S.nterms - P.nterms;
    evals += de;
    const FlopModel &f = set->flops[t];
    flops += f.pre * de + f.post * dp + f.per_term * dt;
  }
  set->last_state = st;
  ctx->evals += evals;
  ctx->flops += flops;
  int status = MBPT_OK;
  mbpt_result tot{};
  double var = 0.0;
  for (int t = 0; t < nt; ++t) {
    mbpt_result r;
    result_of(st[t], r);
    if (!std::isfinite(r.E_per_A) || !std::isfinite(r.sigma)) status = MBPT_ENUMERIC;
    if (per_task) per_task[t] = r;
    tot.E_per_A += r.E_per_A;
    var += r.sigma * r.sigma;
    tot.last_E += r.last_E;
    tot.n_evals += r.n_evals;
    tot.n_fp64_fallback += r.n_fp64_fallback;
    tot.iters_done = std::max(tot.iters_done, r.iters_done);
    tot.chi2_dof = std::max(tot.chi2_dof, r.chi2_dof);
  }
  tot.sigma = std::sqrt(var);
  if (total) *total = tot;
  if (status) set_err(ctx, "integrate: non-finite estimate");
  return status;
}

extern "C" int mbpt_batch_workspace_query(mbpt_context *ctx, const mbpt_task_desc *tasks,
                                          int n_tasks, uint64_t samples_per_iter, int iters,
                                          size_t *bytes) {
  if (!ctx || !tasks || n_tasks < 1 || !bytes) return MBPT_EINVAL;
  mbpt_task_set *set = nullptr;
  int rc = mbpt_create_task_set(ctx, tasks, n_tasks, &set);
  if (rc) return rc;
  rc = mbpt_workspace_query(set, samples_per_iter, iters, bytes);
  mbpt_task_set_destroy(set);
  return rc;
}

extern "C" int mbpt_integrate_batch(mbpt_context *ctx, const mbpt_task_desc *tasks, int n_tasks,
                                    uint64_t samples_per_iter, int iters, void *device_ptr,
                                    size_t bytes, mbpt_result *out, mbpt_result *total) {
  if (!ctx || !tasks || n_tasks < 1) return MBPT_EINVAL;
  mbpt_task_set *set = nullptr;
  int rc = mbpt_create_task_set(ctx, tasks, n_tasks, &set);
  if (rc) return rc;
  rc = mbpt_set_launch_mode(set, MBPT_LAUNCH_BATCHED);
  if (!rc) rc = mbpt_bind_workspace(set, device_ptr, bytes, samples_per_iter, iters);
  if (!rc) rc = mbpt_integrate(set, samples_per_iter, iters, out, total);
  mbpt_task_set_destroy(set);
  return rc;
}

namespace mbpt {

// mbpt_integrate for a set without a workspace, inside device memory the
// caller supplies for this call only: bind (uploads the descriptors and
// parameters, starts every task from a uniform grid at iteration 0), run
// without graph capture or timing events, then leave the set unbound.
int integrate_in(mbpt_task_set *set, void *base, size_t bytes, uint64_t samples_per_iter,
                 int iters, mbpt_result *per_task, mbpt_result *total) {
  if (!set || !base || iters < 1 || samples_per_iter < 2) return MBPT_EINVAL;
  mbpt_context *ctx = set->ctx;
  if (set->ws) {
    set_err(ctx, "integrate_noalloc: the set has a workspace bound (use mbpt_integrate)");
    return MBPT_ESTATE;
  }
  const size_t need = layout_of(set, samples_per_iter, iters, ctx->desc.n_bins).total;
  if (need > bytes) {
    set_err(ctx, "integrate_noalloc: " + std::to_string(set->tasks.size()) + " tasks at " +
                     std::to_string(samples_per_iter) + " samples per iteration and " +
                     std::to_string(iters) + " iterations need " + std::to_string(need) +
                     " bytes of device scratch, more than the " + std::to_string(bytes) +
                     " bytes available");
    return MBPT_ENOMEM;
  }
  int rc = bind(set, base, bytes, samples_per_iter, iters);
  if (rc == MBPT_OK) {
    set->noalloc = true;
    rc = mbpt_integrate(set, samples_per_iter, iters, per_task, total);
    set->noalloc = false;
  }
  set->drop_graph();
  set->ws = nullptr;
  set->ws_bytes = 0;
  set->max_samples = 0;
  set->max_iters = 0;
  set->max_items = 0;
  set->d_tasks = nullptr;
  set->d_olist = nullptr;
  set->d_diags = nullptr;
  set->d_groups = nullptr;
  set->d_terms = nullptr;
  set->d_coefs = nullptr;
  set->d_grids = set->d_hists = set->d_partials = set->d_reslog = nullptr;
  set->d_cpart = set->d_creslog = nullptr;
  set->d_queue = nullptr;
  set->d_counters = nullptr;
  set->d_hf = set->d_gl = nullptr;
  set->hf_dirty = true;
  set->oranges.clear();
  set->last_state.clear();
  set->run_reg_n = -1;
  return rc;
}

}  // namespace mbpt

extern "C" int mbpt_iteration_log(mbpt_task_set *set, int task, double *I, double *var, int cap,
                                  int *count) {
  if (!set || !count || task < 0 || task >= static_cast<int>(set->tasks.size())) return MBPT_EINVAL;
  if (!set->ws) return MBPT_ESTATE;
  mbpt_context *ctx = set->ctx;
  TaskDev S;
  HIPCHK(ctx, hipMemcpyAsync(&S, set->d_tasks + task, sizeof(TaskDev), hipMemcpyDeviceToHost,
                             ctx->stream));
  std::vector<double> lg(2 * set->max_iters);
  HIPCHK(ctx, hipMemcpyAsync(lg.data(), set->d_reslog + 2 * static_cast<size_t>(task) * set->max_iters,
                             lg.size() * sizeof(double), hipMemcpyDeviceToHost, ctx->stream));
  HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
  const int n = std::min(std::min(S.it_done, set->max_iters), cap);
  const int start = S.it_done - n;  // oldest stored iteration that fits
  for (int k = 0; k < n; ++k) {
    const int slot = (start + k) % set->max_iters;
    if (I) I[k] = lg[2 * slot];
    if (var) var[k] = lg[2 * slot + 1];
  }
  *count = n;
  return MBPT_OK;
}

extern "C" int mbpt_dump_samples(mbpt_task_set *set, int task, uint32_t iter, uint64_t first,
                                 uint64_t count, double *w_host) {
  if (!set || !w_host || task < 0 || task >= static_cast<int>(set->tasks.size())) return MBPT_EINVAL;
  if (!set->ws) return MBPT_ESTATE;
  mbpt_context *ctx = set->ctx;
  {
    const int rc = sync_epoch(set);
    if (rc) return rc;
  }
  {
    const int rc = ensure_hf(set);
    if (rc) return rc;
  }
  KArgs a = kargs_of(set);
  // the item partials region serves as staging
  const uint64_t cap = set->max_items * 4;
  for (uint64_t done = 0; done < count;) {
    const uint64_t n = std::min<uint64_t>(cap, count - done);
    HIPCHK(ctx, launch_dump(a, task, set->tasks[task].order, set->q, ctx->desc.precision,
                            set->task_ndiag[task] > 1, iter,
                            first + done, n, set->d_partials, nullptr, ctx->stream));
    HIPCHK(ctx, hipMemcpyAsync(w_host + done, set->d_partials, n * sizeof(double),
                               hipMemcpyDeviceToHost, ctx->stream));
    HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
    done += n;
  }
  return MBPT_OK;
}

extern "C" int mbpt_dump_samples_reg(mbpt_task_set *set, int task, uint32_t iter, uint64_t first,
                                     uint64_t count, double *wreg_host) {
  if (!set || !wreg_host || task < 0 || task >= static_cast<int>(set->tasks.size()))
    return MBPT_EINVAL;
  if (!set->ws) return MBPT_ESTATE;
  mbpt_context *ctx = set->ctx;
  const int K = ctx->reg_n;
  if (K < 1 || ctx->desc.spectrum != MBPT_SPECTRUM_FREE) {
    set_err(ctx, "dump_samples_reg: needs regularised components and the free spectrum");
    return MBPT_ESTATE;
  }
  {
    const int rc = sync_epoch(set);
    if (rc) return rc;
  }
  KArgs a = kargs_of(set);
  // staging: main weights in the item partials, components in the item
  // component sums (kRegSums doubles per item)
  const uint64_t cap = set->max_items * 2;
  for (uint64_t done = 0; done < count;) {
    const uint64_t n = std::min<uint64_t>(cap, count - done);
    HIPCHK(ctx, launch_dump(a, task, set->tasks[task].order, set->q, ctx->desc.precision,
                            set->task_ndiag[task] > 1, iter, first + done, n, set->d_partials,
                            set->d_cpart, ctx->stream));
    HIPCHK(ctx, hipMemcpyAsync(wreg_host + done * K, set->d_cpart, n * K * sizeof(double),
                               hipMemcpyDeviceToHost, ctx->stream));
    HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
    done += n;
  }
  return MBPT_OK;
}

extern "C" int mbpt_regularized_log(mbpt_task_set *set, int task, double *I, double *var, int cap,
                                    int *count) {
  if (!set || !count || task < 0 || task >= static_cast<int>(set->tasks.size())) return MBPT_EINVAL;
  if (!set->ws) return MBPT_ESTATE;
  mbpt_context *ctx = set->ctx;
  const int K = set->run_reg_n > 0 ? set->run_reg_n : 0;
  TaskDev S;
  HIPCHK(ctx, hipMemcpyAsync(&S, set->d_tasks + task, sizeof(TaskDev), hipMemcpyDeviceToHost,
                             ctx->stream));
  const size_t per = kRegSums;
  std::vector<double> lg(per * set->max_iters);
  HIPCHK(ctx, hipMemcpyAsync(lg.data(), set->d_creslog + per * task * set->max_iters,
                             lg.size() * sizeof(double), hipMemcpyDeviceToHost, ctx->stream));
  HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
  const int n = K > 0 ? std::min(std::min(S.it_done, set->max_iters), cap) : 0;
  const int start = S.it_done - n;
  // columns: components 1..K, then the extrapolation (last pair of a log entry)
  for (int i = 0; i < n; ++i) {
    const int slot = (start + i) % set->max_iters;
    for (int k = 0; k <= K; ++k) {
      const int r = k < K ? k : kMaxReg;
      if (I) I[i * (K + 1) + k] = lg[per * slot + 2 * r];
      if (var) var[i * (K + 1) + k] = lg[per * slot + 2 * r + 1];
    }
  }
  *count = n;
  return MBPT_OK;
}

namespace mbpt {

// Weighted least squares of y_k = E_k against polynomials in eta_k of degree
// deg (normal equations, at most 3 x 3, solved by Gaussian elimination with
// partial pivoting); returns the constant term and its standard error from
// the diagonal weights 1 / sigma_k^2.
bool poly_fit_at_zero(const double *x, const double *y, const double *sig, int n, int deg,
                      double &c0, double &s0) {
  const int m = deg + 1;
  double A[3][4] = {};
  for (int k = 0; k < n; ++k) {
    const double w = 1.0 / (sig[k] * sig[k]);
    double pi[3] = {1.0, x[k], x[k] * x[k]};
    for (int i = 0; i < m; ++i) {
      for (int j = 0; j < m; ++j) A[i][j] += w * pi[i] * pi[j];
      A[i][m] += w * pi[i] * y[k];
    }
  }
  // inverse of the normal matrix (for the variance of c0) by Gauss-Jordan
  double M[3][6] = {};
  for (int i = 0; i < m; ++i) {
    for (int j = 0; j < m; ++j) M[i][j] = A[i][j];
    M[i][m + i] = 1.0;
  }
  for (int c = 0; c < m; ++c) {
    int p = c;
    for (int r = c + 1; r < m; ++r)
      if (std::fabs(M[r][c]) > std::fabs(M[p][c])) p = r;
    if (!(std::fabs(M[p][c]) > 0.0)) return false;
    for (int j = 0; j < 2 * m; ++j) std::swap(M[c][j], M[p][j]);
    const double d = M[c][c];
    for (int j = 0; j < 2 * m; ++j) M[c][j] /= d;
    for (int r = 0; r < m; ++r) {
      if (r == c) continue;
      const double f = M[r][c];
      for (int j = 0; j < 2 * m; ++j) M[r][j] -= f * M[c][j];
    }
  }
  c0 = 0.0;
  for (int j = 0; j < m; ++j) c0 += M[0][m + j] * A[j][m];
  s0 = std::sqrt(std::max(0.0, M[0][m]));
  return true;
}

// Weights a_k of the extrapolation to zero shift: the equal-weight
// least-squares polynomial of degree min(2, K - 1) through (k, y_k), k = 1..K,
// takes the value sum_k a_k y_k at 0 (a_k = that value for y = the k-th unit
// vector; the shift's scale drops out).  Zero beyond K.
void extrapolation_weights(int K, double *a) {
  double x[kMaxReg], ones[kMaxReg], e[kMaxReg];
  for (int k = 0; k < kMaxReg; ++k) {
    x[k] = k + 1.0;
    ones[k] = 1.0;
    a[k] = 0.0;
  }
  for (int k = 0; k < K; ++k) {
    for (int j = 0; j < K; ++j) e[j] = j == k ? 1.0 : 0.0;
    double c0 = 0.0, s0 = 0.0;
    if (poly_fit_at_zero(x, e, ones, K, std::min(2, K - 1), c0, s0)) a[k] = c0;
  }
}

}  // namespace mbpt

extern "C" int mbpt_regularized(mbpt_task_set *set, int task, int skip_iters, double *E,
                                double *sigma, double *E0, double *sigma0) {
  if (!set || task < 0 || task >= static_cast<int>(set->tasks.size()) || skip_iters < 0)
    return MBPT_EINVAL;
  if (!set->ws) return MBPT_ESTATE;
  mbpt_context *ctx = set->ctx;
  const int K = set->run_reg_n;
  if (K < 1) {
    set_err(ctx, "regularized: no iterations with regularised components since the last reset");
    return MBPT_ESTATE;
  }
  std::vector<double> I(static_cast<size_t>(set->max_iters) * (K + 1)), V(I.size());
  int n = 0;
  const int rc = mbpt_regularized_log(set, task, I.data(), V.data(), set->max_iters, &n);
  if (rc) return rc;
  // components 1..K, then the extrapolation (column K), each combined over
  // the iterations from skip_iters on by inverse variance
  for (int k = 0; k <= K; ++k) {
    double w = 0.0, wi = 0.0;
    for (int i = skip_iters; i < n; ++i) {
      const double v = V[static_cast<size_t>(i) * (K + 1) + k];
      if (v > 0.0) {
        w += 1.0 / v;
        wi += I[static_cast<size_t>(i) * (K + 1) + k] / v;
      }
    }
    if (!(w > 0.0)) {
      set_err(ctx, "regularized: no iteration with a positive variance after the skipped ones");
      return MBPT_ESTATE;
    }
    const double Ek = wi / w, Sk = 1.0 / std::sqrt(w);
    if (k < K) {
      if (E) E[k] = Ek;
      if (sigma) sigma[k] = Sk;
    } else {
      if (E0) *E0 = Ek;
      if (sigma0) *sigma0 = Sk;
    }
  }
  return MBPT_OK;
}

extern "C" int mbpt_hf_nodes(mbpt_task_set *set, int task, int tau, double *sigma_host,
                             double *h) {
  if (!set || !sigma_host || task < 0 || task >= static_cast<int>(set->tasks.size()) ||
      tau < 0 || tau > (set->q == 4 ? 1 : 0))
    return MBPT_EINVAL;
  mbpt_context *ctx = set->ctx;
  if (!set->ws || ctx->desc.spectrum != MBPT_SPECTRUM_HF) {
    set_err(ctx, "hf_nodes: needs the HF spectrum and a bound workspace");
    return MBPT_ESTATE;
  }
  {
    const int rc = sync_epoch(set);
    if (rc) return rc;
  }
  int rc = ensure_hf(set);
  if (rc) return rc;
  const TaskDev &T = set->h_tasks[task];
  const double *src = set->d_hf + 4 * static_cast<size_t>(T.hf_off + tau * kHfEntries);
  HIPCHK(ctx, hipMemcpy2DAsync(sigma_host, sizeof(double), src, 4 * sizeof(double),
                               sizeof(double), kHfEntries, hipMemcpyDeviceToHost, ctx->stream));
  HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
  if (h) *h = T.hf_h;
  return MBPT_OK;
}

extern "C" int mbpt_get_grid(mbpt_task_set *set, int task, double *edges_host) {
  if (!set || !edges_host || task < 0 || task >= static_cast<int>(set->tasks.size()))
    return MBPT_EINVAL;
  if (!set->ws) return MBPT_ESTATE;
  mbpt_context *ctx = set->ctx;
  const TaskDev &T = set->h_tasks[task];
  HIPCHK(ctx, hipMemcpyAsync(edges_host, set->d_grids + T.grid_off,
                             T.nd * (ctx->desc.n_bins + 1) * sizeof(double), hipMemcpyDeviceToHost,
                             ctx->stream));
  HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
  return MBPT_OK;
}

extern "C" int mbpt_set_grid(mbpt_task_set *set, int task, const double *edges_host) {
  if (!set || !edges_host || task < 0 || task >= static_cast<int>(set->tasks.size()))
    return MBPT_EINVAL;
  if (!set->ws) return MBPT_ESTATE;
  mbpt_context *ctx = set->ctx;
  const TaskDev &T = set->h_tasks[task];
  const int nb = ctx->desc.n_bins;
  for (int m = 0; m < T.nd; ++m) {
    const double *e = edges_host + m * (nb + 1);
    if (e[0] != 0.0 || e[nb] != 1.0) return MBPT_EINVAL;
    for (int b = 0; b < nb; ++b)
      if (!(e[b + 1] > e[b])) return MBPT_EINVAL;
  }
  HIPCHK(ctx, hipMemcpyAsync(set->d_grids + T.grid_off, edges_host,
                             T.nd * (nb + 1) * sizeof(double), hipMemcpyHostToDevice, ctx->stream));
  HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
  return MBPT_OK;
}

extern "C" int mbpt_kernel_stats(mbpt_context *ctx, uint64_t *launches, double *kernel_ms,
                                 uint64_t *evals, double *flops) {
  if (!ctx) return MBPT_EINVAL;
  if (launches) *launches = ctx->launches;
  if (kernel_ms) *kernel_ms = ctx->kernel_ms;
  if (evals) *evals = ctx->evals;
  if (flops) *flops = ctx->flops;
  ctx->launches = 0;
  ctx->kernel_ms = 0.0;
  ctx->evals = 0;
  ctx->flops = 0.0;
  return MBPT_OK;
}

extern "C" int mbpt_diagram_flops(int order, int id, int matter, int label_mode, int reg_exp,
                                  int spectrum, double *pre, double *post, double *per_unit,
                                  double *units) {
  const Diagram *d = get_diagram(order, id);
  if (!d || (matter != MBPT_NEUTRON && matter != MBPT_NUCLEAR) || (label_mode & ~1) ||
      reg_exp < 2 || reg_exp > 16 || (reg_exp & 1) || (spectrum & ~1))
    return MBPT_EINVAL;
  const int q = matter == MBPT_NUCLEAR ? 4 : 2;
  FlopModel f;
  count_flops(*d, q, reg_exp / 2, label_mode, spectrum, f);
  const LabelTables lt = label_tables(*d, q);
  if (pre) *pre = f.pre;
  if (post) *post = f.post;
  if (per_unit) *per_unit = f.per_term;
  if (units)
    *units = static_cast<double>(label_mode ? lt.terms.size()
                                 : (q == 4 && spectrum == MBPT_SPECTRUM_FREE) ? 1
                                                                              : lt.groups.size());
  return MBPT_OK;
}

extern "C" int mbpt_task_flops(const mbpt_task_set *set, int task, double *flops,
                               double *transcendentals) {
  if (!set || task < 0 || task >= static_cast<int>(set->tasks.size())) return MBPT_EINVAL;
  const FlopModel &f = set->flops[task];
  if (flops) *flops = f.pre + f.post + f.per_term * f.all_units;
  if (transcendentals) *transcendentals = f.transc_pre + f.transc_post;
  return MBPT_OK;
}

// ---------------------------------------------------------------------------
// Autotuner

namespace {
struct TuneKey {
  int q, prec, mode;
  uint32_t orders;  // bit k: order k present
  uint64_t samples;
  bool operator<(const TuneKey &o) const {
    return std::tie(q, prec, mode, orders, samples) < std::tie(o.q, o.prec, o.mode, o.orders, o.samples);
  }
};
std::map<TuneKey, std::pair<int, int>> &tune_cache() {
  static std::map<TuneKey, std::pair<int, int>> c;
  return c;
}
}  // namespace

extern "C" int mbpt_autotune(mbpt_task_set *set, uint64_t samples_per_iter, int *threads_per_block,
                             int *samples_per_thread, double *ms_per_iter) {
  if (!set || samples_per_iter < 2) return MBPT_EINVAL;
  mbpt_context *ctx = set->ctx;
  if (!set->ws) {
    set_err(ctx, "autotune: no workspace bound");
    return MBPT_ESTATE;
  }
  if (samples_per_iter > set->max_samples) return MBPT_ENOMEM;
  TuneKey key{set->q, ctx->desc.precision, set->launch_mode, 0u, samples_per_iter};
  for (const auto &t : set->tasks) key.orders |= 1u << t.order;
  const int old_block = set->block, old_spt = set->spt;
  int best_b = old_block, best_s = old_spt;
  double best_ms = -1.0;
  // the workspace holds items for the bind-time shape: only shapes with
  // work items at least that large fit
  const size_t bound_chunk = set->max_items / std::max<size_t>(1, set->tasks.size());
  auto fits = [&](int b, int sp) {
    set->block = b;
    set->spt = sp;
    const bool ok = items_for(set, samples_per_iter) <= bound_chunk;
    set->block = old_block;
    set->spt = old_spt;
    return ok;
  };
  auto it = tune_cache().find(key);
  if (it != tune_cache().end() && fits(it->second.first, it->second.second)) {
    // a shape tuned on another workspace applies only if this one holds it
    best_b = it->second.first;
    best_s = it->second.second;
  } else {
    const int blocks[] = {64, 128, 256};
    const int spts[] = {4, 8, 16, 32, 64, 128, 256};
    bool warmed = false;
    for (int b : blocks)
      for (int sp : spts) {
        set->block = b;
        set->spt = sp;
        set->oranges.clear();
        if (items_for(set, samples_per_iter) > bound_chunk) continue;
        set->drop_graph();
        const int saved_mode = set->launch_mode;
        if (set->launch_mode == MBPT_LAUNCH_GRAPH) set->launch_mode = MBPT_LAUNCH_BATCHED;
        uint64_t l0;
        double ms0;
        mbpt_kernel_stats(ctx, &l0, &ms0, nullptr, nullptr);  // drain earlier stats
        const uint64_t ev = ctx->evals;
        const double fl = ctx->flops;
        int rc = 0;
        if (!warmed) {
          rc = mbpt_integrate(set, samples_per_iter, 1, nullptr, nullptr);
          warmed = true;
        }
        if (!rc) rc = mbpt_integrate(set, samples_per_iter, 1, nullptr, nullptr);
        set->launch_mode = saved_mode;
        uint64_t launches;
        double ms;
        mbpt_kernel_stats(ctx, &launches, &ms, nullptr, nullptr);
        ctx->evals = ev;
        ctx->flops = fl;
        if (rc && rc != MBPT_ENUMERIC) return rc;
        if (best_ms < 0.0 || ms < best_ms) {
          best_ms = ms;
          best_b = b;
          best_s = sp;
        }
      }
    tune_cache()[key] = {best_b, best_s};
  }
  set->block = best_b;
  set->spt = best_s;
  set->oranges.clear();
  set->drop_graph();
  const int rc = mbpt_reset(set);
  if (rc) return rc;
  if (threads_per_block) *threads_per_block = best_b;
  if (samples_per_thread) *samples_per_thread = best_s;
  if (ms_per_iter) *ms_per_iter = best_ms;
  return MBPT_OK;
}
