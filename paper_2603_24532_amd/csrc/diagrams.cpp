// Diagram generator and descriptor compiler (host side).  See diagrams.hpp.
#include "diagrams.hpp"

#include <algorithm>
#include <array>
#include <cmath>
#include <map>
#include <mutex>
#include <string>

namespace mbpt {
namespace {

using Mat = std::array<int, kMaxOrder * kMaxOrder>;

// Fill the off-diagonal entries of an n x n matrix with values in {0,1,2} so
// that every row and every column sums to 2.
void fill(int n, int pos, Mat &m, int *row_left, int *col_left, std::vector<Mat> &out) {
  if (pos == n * n) {
    for (int i = 0; i < n; ++i)
      if (row_left[i] || col_left[i]) return;
    out.push_back(m);
    return;
  }
  const int u = pos / n, v = pos % n;
  if (v == 0 && u > 0 && row_left[u - 1]) return;  // previous row incomplete
  if (u == v) {
    fill(n, pos + 1, m, row_left, col_left, out);
    return;
  }
  const int hi = std::min(row_left[u], col_left[v]);
  for (int val = 0; val <= hi; ++val) {
    m[u * kMaxOrder + v] = val;
    row_left[u] -= val;
    col_left[v] -= val;
    fill(n, pos + 1, m, row_left, col_left, out);
    row_left[u] += val;
    col_left[v] += val;
  }
  m[u * kMaxOrder + v] = 0;
}

bool is_connected(int n, const Mat &m) {
  int comp[kMaxOrder];
  for (int i = 0; i < n; ++i) comp[i] = i;
  bool changed = true;
  while (changed) {  // propagate the smallest label along edges
    changed = false;
    for (int u = 0; u < n; ++u)
      for (int v = 0; v < n; ++v)
        if (u != v && m[u * kMaxOrder + v] > 0) {
          int lo = std::min(comp[u], comp[v]);
          if (comp[u] != lo || comp[v] != lo) {
            comp[u] = comp[v] = lo;
            changed = true;
          }
        }
  }
  for (int i = 0; i < n; ++i)
    if (comp[i] != 0) return false;
  return true;
}

std::vector<Mat> enumerate(int n) {
  std::vector<Mat> all;
  if (n == 1) {
    Mat m{};
    m[0] = 2;  // one vertex, two hole self-lines
    all.push_back(m);
    return all;
  }
  Mat m{};
  int rl[kMaxOrder], cl[kMaxOrder];
  for (int i = 0; i < n; ++i) rl[i] = cl[i] = 2;
  fill(n, 0, m, rl, cl, all);
  std::vector<Mat> conn;
  for (auto &x : all)
    if (is_connected(n, x)) conn.push_back(x);
  auto key = [n](const Mat &a) {
    std::array<int, kMaxOrder * kMaxOrder> k{};
    for (int u = 0; u < n; ++u)
      for (int v = 0; v < n; ++v) k[u * n + v] = a[u * kMaxOrder + v];
    return k;
  };
  std::sort(conn.begin(), conn.end(), [&](const Mat &a, const Mat &b) { return key(a) < key(b); });
  return conn;
}

void compile(int n, int id, const Mat &m, Diagram &d) {
  d.order = n;
  d.id = id;
  for (int u = 0; u < n; ++u)
    for (int v = 0; v < n; ++v) d.M[u][v] = m[u * kMaxOrder + v];
  // lines: particles (u < v) in lexicographic (u, v) order, then holes
  int nl = 0;
  for (int pass = 0; pass < 2; ++pass)
    for (int u = 0; u < n; ++u)
      for (int v = 0; v < n; ++v) {
        const bool part = u < v;
        const bool hole = u > v || (n == 1 && u == v);
        if ((pass == 0 && !part) || (pass == 1 && !hole)) continue;
        for (int c = 0; c < d.M[u][v]; ++c) {
          d.tail[nl] = u;
          d.head[nl] = v;
          d.particle[nl] = part;
          ++nl;
        }
      }
  d.nlines = nl;
  d.nloops = n + 1;
  d.ncuts = n - 1;
  d.ndim = 3 * d.nloops;
  for (int v = 0; v < n; ++v) {
    int no = 0, ni = 0;
    for (int l = 0; l < nl; ++l) {
      if (d.tail[l] == v) d.vout[v][no++] = l;
      if (d.head[l] == v) d.vin[v][ni++] = l;
    }
  }
  // prefactor: (1/2)^{equivalent pairs} (-1)^{holes + closed loops}
  d.n_h = 0;
  for (int l = 0; l < nl; ++l) d.n_h += d.particle[l] ? 0 : 1;
  d.n_eq = n == 1 ? 1 : 0;
  for (int u = 0; u < n; ++u)
    for (int v = 0; v < n; ++v)
      if (u != v && d.M[u][v] == 2) ++d.n_eq;
  {
    bool seen[kMaxLines] = {};
    d.n_cycles = 0;
    for (int s = 0; s < nl; ++s) {
      if (seen[s]) continue;
      ++d.n_cycles;
      for (int l = s; !seen[l];) {
        seen[l] = true;
        const int v = d.head[l];
        l = d.vout[v][d.vin[v][0] == l ? 0 : 1];  // in slot k continues as out slot k
      }
    }
  }
  d.prefactor = ((d.n_h + d.n_cycles) & 1 ? -1.0 : 1.0);
  for (int i = 0; i < d.n_eq; ++i) d.prefactor *= 0.5;

  // loop lines: scan lines in order, a line joining two already-connected
  // vertex sets closes a loop and carries a loop momentum
  bool tree[kMaxLines] = {};
  {
    int comp[kMaxOrder];
    for (int v = 0; v < n; ++v) comp[v] = v;
    int nloop = 0;
    for (int l = 0; l < nl; ++l) {
      const int a = comp[d.tail[l]], b = comp[d.head[l]];
      if (a == b) {
        d.loop_line[nloop++] = l;
      } else {
        tree[l] = true;
        for (int v = 0; v < n; ++v)
          if (comp[v] == b) comp[v] = a;
      }
    }
  }
  // routing: loop lines are unit vectors; tree lines are solved leaf by leaf
  // from momentum conservation (sum in = sum out) at each vertex
  bool known[kMaxLines] = {};
  for (int j = 0; j < d.nloops; ++j) {
    known[d.loop_line[j]] = true;
    d.coef[d.loop_line[j]][j] = 1;
  }
  for (int solved = 0; solved < n - 1;) {
    bool progress = false;
    for (int v = 0; v < n && !progress; ++v) {
      int unknown = -1, cnt = 0;
      for (int l = 0; l < nl; ++l)
        if ((d.tail[l] == v || d.head[l] == v) && !known[l]) {
          unknown = l;
          ++cnt;
        }
      if (cnt != 1) continue;
      int acc[kMaxLoops] = {};
      // k_unknown = (momenta flowing the other way) - (same way, others)
      const int sgn_in = d.head[unknown] == v ? 1 : -1;
      for (int l = 0; l < nl; ++l) {
        if (l == unknown) continue;
        int s = 0;
        if (d.head[l] == v) s -= sgn_in;
        if (d.tail[l] == v) s += sgn_in;
        for (int j = 0; j < d.nloops; ++j) acc[j] += s * d.coef[l][j];
      }
      for (int j = 0; j < d.nloops; ++j) d.coef[unknown][j] = acc[j];
      known[unknown] = true;
      ++solved;
      progress = true;
    }
    if (!progress) break;
  }
  for (int c = 0; c < d.ncuts; ++c)
    for (int l = 0; l < nl; ++l) {
      const int lo = std::min(d.tail[l], d.head[l]), hi = std::max(d.tail[l], d.head[l]);
      d.cut[c][l] = (lo <= c && c < hi) ? (d.particle[l] ? -1 : 1) : 0;
    }
}

struct Cache {
  std::mutex mu;
  std::map<int, std::vector<Diagram>> by_order;
};
Cache &cache() {
  static Cache c;
  return c;
}

const std::vector<Diagram> &diagrams_of(int order) {
  Cache &c = cache();
  std::lock_guard<std::mutex> lk(c.mu);
  auto it = c.by_order.find(order);
  if (it != c.by_order.end()) return it->second;
  std::vector<Mat> mats = enumerate(order);
  std::vector<Diagram> ds(mats.size());
  for (size_t i = 0; i < mats.size(); ++i) compile(order, static_cast<int>(i), mats[i], ds[i]);
  return c.by_order.emplace(order, std::move(ds)).first->second;
}

// Depth-first label assignment with a vertex check as soon as all four of a
// vertex's lines carry labels.
struct LabelSearch {
  const Diagram &d;
  int q;
  int lab[kMaxLines];
  int last_line_of_vertex[kMaxOrder];
  std::map<std::pair<uint32_t, uint32_t>, int> patterns;
  std::map<uint32_t, int> iso;
  int n_assign = 0;

  LabelSearch(const Diagram &dd, int qq) : d(dd), q(qq) {
    for (int v = 0; v < d.order; ++v)
      last_line_of_vertex[v] = std::max(std::max(d.vout[v][0], d.vout[v][1]),
                                        std::max(d.vin[v][0], d.vin[v][1]));
  }
  bool vertex_ok(int v) const {
    const int o1 = lab[d.vout[v][0]], o2 = lab[d.vout[v][1]];
    const int i1 = lab[d.vin[v][0]], i2 = lab[d.vin[v][1]];
    return (o1 == i1 && o2 == i2) || (o1 == i2 && o2 == i1);
  }
  void rec(int l) {
    if (l == d.nlines) {
      uint32_t codes = 0, tau = 0;
      for (int v = 0; v < d.order; ++v) {
        const int o1 = lab[d.vout[v][0]], o2 = lab[d.vout[v][1]];
        const int i1 = lab[d.vin[v][0]], i2 = lab[d.vin[v][1]];
        const bool dir = o1 == i1 && o2 == i2, exc = o1 == i2 && o2 == i1;
        const uint32_t code = dir && exc ? 2u : (dir ? 0u : 1u);
        codes |= code << (2 * v);
      }
      for (int k = 0; k < d.nlines; ++k)
        if (q == 4 && (lab[k] >> 1)) tau |= 1u << k;
      ++patterns[{tau, codes}];
      ++iso[tau];
      ++n_assign;
      return;
    }
    for (int x = 0; x < q; ++x) {
      lab[l] = x;
      bool ok = true;
      for (int v = 0; v < d.order && ok; ++v)
        if (last_line_of_vertex[v] == l) ok = vertex_ok(v);
      if (ok) rec(l + 1);
    }
  }
};

}  // namespace

int num_diagrams(int order) {
  if (order < 1 || order > kMaxOrder) return -1;
  return static_cast<int>(diagrams_of(order).size());
}

const Diagram *get_diagram(int order, int id) {
  if (order < 1 || order > kMaxOrder) return nullptr;
  const auto &ds = diagrams_of(order);
  if (id < 0 || id >= static_cast<int>(ds.size())) return nullptr;
  return &ds[id];
}

int diagram_from_lines(int order, int nlines, const int *from, const int *to,
                       const int (*vertex)[4], std::string &err) {
  if (order < 1 || order > kMaxOrder) {
    err = "order must be 1..5";
    return -1;
  }
  if (nlines != 2 * order) {
    err = "an order-n two-body energy diagram has 2n lines";
    return -1;
  }
  Mat m{};
  int nout[kMaxOrder] = {}, nin[kMaxOrder] = {};
  for (int l = 0; l < nlines; ++l) {
    const int u = from[l], v = to[l];
    if (u < 0 || u >= order || v < 0 || v >= order) {
      err = "line " + std::to_string(l) + ": level outside 0..order-1";
      return -1;
    }
    if (u == v && order > 1) {
      err = "line " + std::to_string(l) + ": self-line above first order";
      return -1;
    }
    ++m[u * kMaxOrder + v];
    ++nout[u];
    ++nin[v];
  }
  for (int v = 0; v < order; ++v) {
    if (nout[v] != 2 || nin[v] != 2) {
      err = "vertex " + std::to_string(v) + ": needs two lines leaving and two entering";
      return -1;
    }
    // outgoing slots name two distinct lines, incoming slots two distinct
    // lines (at first order the two self-lines fill both pairs)
    bool used[2][kMaxLines] = {};
    for (int s = 0; s < 4; ++s) {
      const int l = vertex[v][s];
      if (l < 0 || l >= nlines || used[s / 2][l]) {
        err = "vertex " + std::to_string(v) + ": o1, o2 and i1, i2 must name distinct lines";
        return -1;
      }
      used[s / 2][l] = true;
      // slots 0, 1 (o1, o2) leave the vertex, slots 2, 3 (i1, i2) enter it
      const bool ok = s < 2 ? from[l] == v : to[l] == v;
      if (!ok) {
        err = "vertex " + std::to_string(v) + ": slot " + std::to_string(s) +
              " names a line that does not " + (s < 2 ? "leave" : "enter") + " it";
        return -1;
      }
    }
  }
  if (order > 1 && !is_connected(order, m)) {
    err = "the lines do not connect all vertices (not a linked energy diagram)";
    return -1;
  }
  const auto &ds = diagrams_of(order);
  for (const auto &d : ds) {
    bool same = true;
    for (int u = 0; u < order && same; ++u)
      for (int v = 0; v < order && same; ++v) same = d.M[u][v] == m[u * kMaxOrder + v];
    if (same) return d.id;
  }
  err = "no generator diagram has these lines";  // unreachable for a valid diagram
  return -1;
}

int particle_loops(const Diagram &d) {
  int p = 0;
  for (int j = 0; j < d.nloops; ++j) p += d.particle[d.loop_line[j]] ? 1 : 0;
  return p;
}

std::vector<int> group_members(int order, int p) {
  std::vector<int> ids;
  const int n = num_diagrams(order);
  for (int i = 0; i < n; ++i) {
    const Diagram *d = get_diagram(order, i);
    if (d && particle_loops(*d) == p) ids.push_back(i);
  }
  return ids;
}

void canonical_loops(const Diagram &d, int *canon) {
  int c = 0;
  for (int j = 0; j < d.nloops; ++j)
    if (d.particle[d.loop_line[j]]) canon[c++] = j;
  for (int j = 0; j < d.nloops; ++j)
    if (!d.particle[d.loop_line[j]]) canon[c++] = j;
}

void line_slots(const Diagram &d, int *slot_line, bool canonical) {
  bool is_loop[kMaxLines] = {};
  int canon[kMaxLoops];
  for (int j = 0; j < d.nloops; ++j) canon[j] = j;
  if (canonical) canonical_loops(d, canon);
  for (int j = 0; j < d.nloops; ++j) {
    slot_line[j] = d.loop_line[canon[j]];
    is_loop[d.loop_line[j]] = true;
  }
  int k = d.nloops;
  for (int l = 0; l < d.nlines; ++l)
    if (!is_loop[l]) slot_line[k++] = l;
}

LabelTables label_tables(const Diagram &d, int q, bool canonical) {
  const LabelList ll = build_labels(d, q);
  int slot_line[kMaxLines];
  line_slots(d, slot_line, canonical);
  auto to_slots = [&](uint32_t tau) {
    uint32_t t = 0;
    for (int sl = 0; sl < d.nlines; ++sl)
      if ((tau >> slot_line[sl]) & 1u) t |= 1u << sl;
    return t;
  };
  LabelTables out;
  std::vector<LabelTerm> terms;
  for (const auto &t : ll.terms) terms.push_back({to_slots(t.tau_mask), t.codes, t.mult});
  std::sort(terms.begin(), terms.end(), [](const LabelTerm &x, const LabelTerm &y) {
    return x.tau_mask != y.tau_mask ? x.tau_mask < y.tau_mask : x.codes < y.codes;
  });
  out.terms = terms;
  const int n = d.order, nE = 1 << n;
  for (size_t i = 0; i < terms.size();) {
    size_t j = i;
    while (j < terms.size() && terms[j].tau_mask == terms[i].tau_mask) ++j;
    LabelTables::Group g;
    g.tau = terms[i].tau_mask;
    g.first = static_cast<int>(i);
    g.count = static_cast<int>(j - i);
    g.coef.assign(nE, 0.0);
    for (size_t t = i; t < j; ++t)
      for (int E = 0; E < nE; ++E) {
        // code 0: V_d (a = 1, b = 0); 1: -V_e (a = 0, b = -1); 2: V_d - V_e (1, -1)
        int c = terms[t].mult;
        for (int v = 0; v < n && c; ++v) {
          const uint32_t code = (terms[t].codes >> (2 * v)) & 3u;
          if ((E >> v) & 1) c *= (code == 0u) ? 0 : -1;
          else c *= (code == 1u) ? 0 : 1;
        }
        g.coef[E] += c;
      }
    out.groups.push_back(std::move(g));
    i = j;
  }
  return out;
}

CycleTables cycle_tables(const Diagram &d, bool canonical) {
  int slot_line[kMaxLines], slot_of[kMaxLines];
  line_slots(d, slot_line, canonical);
  for (int sl = 0; sl < d.nlines; ++sl) slot_of[slot_line[sl]] = sl;
  CycleTables out;
  const int n = d.order, nE = 1 << n;
  for (int E = 0; E < nE; ++E) {
    int root[kMaxLines];
    for (int l = 0; l < d.nlines; ++l) root[l] = l;
    auto find = [&](int x) {
      while (root[x] != x) x = root[x] = root[root[x]];
      return x;
    };
    for (int v = 0; v < n; ++v) {
      const int o1 = d.vout[v][0], o2 = d.vout[v][1];
      const int i1 = d.vin[v][0], i2 = d.vin[v][1];
      const bool ex = (E >> v) & 1;
      root[find(o1)] = find(ex ? i2 : i1);
      root[find(o2)] = find(ex ? i1 : i2);
    }
    uint32_t comp[kMaxLines] = {};
    for (int l = 0; l < d.nlines; ++l) comp[find(l)] |= 1u << slot_of[l];
    uint64_t bits = 0;
    int count = 0;
    for (int l = 0; l < d.nlines; ++l) {
      if (!comp[l]) continue;
      ++count;
      size_t k = 0;
      while (k < out.masks.size() && out.masks[k] != comp[l]) ++k;
      if (k == out.masks.size()) out.masks.push_back(comp[l]);
      bits |= uint64_t{1} << k;
    }
    out.of_e.push_back(bits);
    out.n_of_e.push_back(count);
  }
  return out;
}

bool cycles_match_label_tables(const Diagram &d, int q, bool canonical) {
  const LabelTables lt = label_tables(d, q, canonical);
  const CycleTables ct = cycle_tables(d, canonical);
  const int nE = 1 << d.order;
  for (const auto &g : lt.groups)
    for (int E = 0; E < nE; ++E) {
      bool constant = true;
      for (size_t k = 0; k < ct.masks.size(); ++k) {
        if (!((ct.of_e[E] >> k) & 1u)) continue;
        const uint32_t t = g.tau & ct.masks[k];
        constant = constant && (t == 0u || t == ct.masks[k]);
      }
      const int sign = __builtin_popcount(static_cast<unsigned>(E)) & 1 ? -1 : 1;
      const double want = constant ? sign * std::ldexp(1.0, ct.n_of_e[E]) : 0.0;
      if (g.coef[E] != want) return false;
    }
  // every isospin pattern constant on some E's cycles is one of the groups
  // (q = 4): count them against the table's groups
  if (q == 4) {
    std::vector<uint32_t> seen;
    for (int E = 0; E < nE; ++E) {
      std::vector<uint32_t> cyc;
      for (size_t k = 0; k < ct.masks.size(); ++k)
        if ((ct.of_e[E] >> k) & 1u) cyc.push_back(ct.masks[k]);
      for (uint32_t pick = 0; pick < (1u << cyc.size()); ++pick) {
        uint32_t tau = 0;
        for (size_t c = 0; c < cyc.size(); ++c)
          if ((pick >> c) & 1u) tau |= cyc[c];
        if (std::find(seen.begin(), seen.end(), tau) == seen.end()) seen.push_back(tau);
      }
    }
    if (seen.size() != lt.groups.size()) return false;
  }
  return true;
}

LabelList build_labels(const Diagram &d, int q) {
  LabelSearch s(d, q);
  s.rec(0);
  LabelList out;
  out.n_assign = s.n_assign;
  out.n_isospin = static_cast<int>(s.iso.size());
  for (const auto &kv : s.patterns) out.terms.push_back({kv.first.first, kv.first.second, kv.second});
  return out;  // std::map order: by tau_mask, then codes
}

}  // namespace mbpt
