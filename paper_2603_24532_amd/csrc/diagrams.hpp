// Diagram generator and descriptor compiler (host side).
//
// Two-body Hugenholtz energy diagrams of order n (Table I of arXiv:2603.24532:
// 1, 1, 3, 39, 840 diagrams for n = 1..5) are enumerated as n x n line-count
// matrices; each is compiled into the tables the sample kernels read:
// line momenta as +-1 combinations of loop momenta, vertex relative momenta,
// energy-denominator cuts, prefactor, and the list of nonzero spin(-isospin)
// label assignments compressed into (isospin pattern, vertex term codes,
// multiplicity) terms.
#pragma once
#include <cstdint>
#include <string>
#include <vector>

namespace mbpt {

constexpr int kMaxOrder = 5;
constexpr int kMaxLines = 2 * kMaxOrder;
constexpr int kMaxLoops = kMaxOrder + 1;
constexpr int kMaxCuts = kMaxOrder - 1;
constexpr int kMaxDim = 3 * kMaxLoops;

struct Diagram {
  int order = 0, id = 0;
  int M[kMaxOrder][kMaxOrder] = {};
  int nlines = 0, nloops = 0, ncuts = 0, ndim = 0;
  int tail[kMaxLines] = {}, head[kMaxLines] = {};
  bool particle[kMaxLines] = {};
  int vout[kMaxOrder][2] = {}, vin[kMaxOrder][2] = {};  // <o1 o2|V|i1 i2>
  int loop_line[kMaxLoops] = {};
  int coef[kMaxLines][kMaxLoops] = {};  // k_line = sum_j coef[line][j] k_loop(j)
  int cut[kMaxCuts][kMaxLines] = {};    // +1 hole crosses, -1 particle crosses
  int n_eq = 0, n_h = 0, n_cycles = 0;
  double prefactor = 0.0;
};

// Vertex term codes of one label assignment: the antisymmetrised matrix
// element <o1 o2|V(1-P12)|i1 i2> with labels is V_d [o1=i1][o2=i2] -
// V_e [o1=i2][o2=i1]; code 0 = V_d only, 1 = -V_e only, 2 = V_d - V_e.
struct LabelTerm {
  uint32_t tau_mask;  // bit l: line l carries a proton label
  uint32_t codes;     // 2 bits per vertex
  int mult;           // number of label assignments with this pattern
};

struct LabelList {
  int n_assign = 0;    // nonzero label assignments
  int n_isospin = 0;   // distinct isospin configurations among them
  std::vector<LabelTerm> terms;  // sorted by tau_mask, then codes
};

// Validates a diagram given by its lines and vertices and returns the
// generator id of the same Hugenholtz diagram, or -1 with `err` set.  Line l
// runs from time level from[l] to level to[l] (particle if from < to, hole if
// from > to; at first order two hole self-lines 0 -> 0); vertex[v] lists the
// line ids of <o1 o2|V|i1 i2> at vertex v (o1, o2 leave it, i1, i2 enter it).
// A two-body energy diagram is fixed by its line-count matrix M[u][v]:
// relabelling its lines, or exchanging a vertex's two incoming lines (which
// flips the antisymmetrised matrix element and the closed-loop count
// together), leaves its value unchanged, so every valid description of a
// matrix maps to the generator's compiled form of that matrix.
int diagram_from_lines(int order, int nlines, const int *from, const int *to,
                       const int (*vertex)[4], std::string &err);

// Loop momenta carried by particle lines (the cycle rank of the particle-line
// subgraph, since the spanning forest takes particle lines first).  Diagrams
// of an order with equal counts form a diagram group; this gives 1, 1, 2, 4, 5
// groups at orders 1..5 (Table I, N_grp).
int particle_loops(const Diagram &d);
// Ids of the diagrams of `order` with p particle-carried loops, ascending.
std::vector<int> group_members(int order, int p);
// Canonical loop order of a group member: its particle loops first, then its
// hole loops, each in the diagram's own order.  canon[c] = the diagram's loop.
void canonical_loops(const Diagram &d, int *canon);

// Line slots: slot j < L holds the line carrying loop momentum j (in the
// canonical order if `canonical`), the tree lines follow in line order.
// slot_line[slot] = line.
void line_slots(const Diagram &d, int *slot_line, bool canonical = false);

// Device-ready label tables of one diagram, with lines in slot order:
// isospin groups (tau masks over slots), explicit terms and, per group, the
// 2^n coefficients c_E of the multilinear expansion
//   sum_{terms} mult prod_v (a_v V_d,v + b_v V_e,v) = sum_E c_E prod_{v not in E} V_d,v prod_{v in E} V_e,v
// (E = set of vertices taking the exchange term; bit v of the index E).
struct LabelTables {
  struct Group {
    uint32_t tau;
    int first, count;
    std::vector<double> coef;
  };
  std::vector<Group> groups;
  std::vector<LabelTerm> terms;  // tau masks over slots
};
LabelTables label_tables(const Diagram &d, int q, bool canonical = false);

// Label cycles of the vertex-term choices E (bit v of E: exchange at vertex
// v).  With the direct term the labels of o1 and i1 and of o2 and i2 are
// equal, with the exchange term those of o1 and i2 and of o2 and i1; every
// line meets two vertex slots, so for each E the lines fall into closed
// cycles of equal labels.  For a spin(-isospin)-independent interaction the
// label sum of E is then (-1)^{|E|} prod_{cycles} (spin states x sum over the
// isospins allowed on every line of the cycle), and the coefficient of E in
// an isospin configuration's polynomial (label_tables) is (-1)^{|E|}
// 2^{cycles(E)} if the configuration is constant on each cycle of E, else 0.
struct CycleTables {
  std::vector<uint32_t> masks;  // distinct cycles as line-slot masks
  std::vector<uint64_t> of_e;   // per E: bit k set if cycle k is one of E's
  std::vector<int> n_of_e;      // per E: its number of cycles
};
CycleTables cycle_tables(const Diagram &d, bool canonical = false);
// True if every coefficient of label_tables(d, q) equals the cycle form above.
bool cycles_match_label_tables(const Diagram &d, int q, bool canonical = false);

// Number of diagrams of an order (1..5), or -1.
int num_diagrams(int order);
// Diagram `id` of an order (ids follow the lexicographic order of the
// row-major matrix digits).  Returns nullptr if out of range.
const Diagram *get_diagram(int order, int id);
// q = 2: spin labels (neutron matter); q = 4: spin x isospin, label bit 1 is
// the isospin (0 neutron, 1 proton).
LabelList build_labels(const Diagram &d, int q);

}  // namespace mbpt
