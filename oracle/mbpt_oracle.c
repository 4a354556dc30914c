/*
 * mbpt_oracle.c -- CPU oracle for VEGAS Monte Carlo evaluation of MBPT
 * (Goldstone/Hugenholtz) energy diagrams of infinite nucleon matter.
 *
 * TEST INFRASTRUCTURE ONLY.  This file is compiled into liboracle.so, which
 * only the test suite, the smoke check and the CPU-baseline leg of the
 * benchmark load.  The product library never links, loads or calls it, and
 * the two share no source, header, table or helper.
 *
 * Everything here is plain, slow, fp64 C written from the definitions:
 *
 *  - Philox4x32-10: Salmon, Moraes, Dror, Shaw, "Parallel random numbers: as
 *    easy as 1, 2, 3" (SC'11).  Pinned against rocRAND's implementation.
 *  - Diagrams: order-n two-body energy diagrams in Hugenholtz form, one per
 *    n x n matrix M (zero diagonal, rows and columns summing to 2, connected),
 *    M[u][v] lines running from time level u to level v (particle if u < v,
 *    hole if u > v).  Counts pinned against Table I of the paper
 *    (N_diag = 1, 1, 3, 39, 840).  Prefactor (1/2)^{n_eq} (-1)^{n_h + n_loop}
 *    pinned against Eqs. (2)-(5) (E_2nd, E_3rd_hh/ph/pp).
 *  - Integrand: sum over hole/particle states with the measure
 *    sum_{sigma tau} int d^3k/(2pi)^3 n_k or (1 - n_k) (shorthand below
 *    Eq. (5)), zero-temperature n_k = theta(kF - k), kF = (3 pi^2 n_tau)^{1/3},
 *    energy denominators D = sum eps_holes - sum eps_particles (equation
 *    eq:Dijkabc), antisymmetrized matrix elements <12|V(1-P12)|34>.  Free
 *    spectrum eps = (hbar^2/2m) k^2.  The spin(-isospin) sum is done by brute
 *    force over all q^{2n} label assignments (the plain definition) or, as a
 *    second form pinned to the first, by the closed-loop (trace) rule.
 *  - VEGAS: Lepage, J. Comput. Phys. 27 (1978) 192 -- piecewise-linear
 *    per-dimension maps, bin histograms of w^2, smoothing + compression with
 *    exponent alpha, inverse-variance combination of iterations (the paper's
 *    Sec. "MC integration: PVegas and Mpi_Jm" builds on this algorithm).
 *
 * Readings where the paper is silent (hypercube -> momentum map, truncation
 * radius of particle loops, uniform -> bin mapping, choice of loop momenta)
 * are fixed rules stated where they are implemented.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORC_MAXN 5
#define ORC_MAXLINES 10
#define ORC_MAXLOOPS 6
#define ORC_MAXCUTS 4
#define ORC_MAXDIM 18
#define ORC_MAXBINS 256

/* ------------------------------------------------------------------------ */
/* Philox4x32-10 (Salmon et al., SC'11)                                      */
/* ------------------------------------------------------------------------ */

void orc_philox4x32_10(const uint32_t ctr_in[4], const uint32_t key_in[2],
                       uint32_t out[4]) {
  const uint32_t M0 = 0xD2511F53u, M1 = 0xCD9E8D57u;
  const uint32_t W0 = 0x9E3779B9u, W1 = 0xBB67AE85u;
  uint32_t c0 = ctr_in[0], c1 = ctr_in[1], c2 = ctr_in[2], c3 = ctr_in[3];
  uint32_t k0 = key_in[0], k1 = key_in[1];
  for (int round = 0; round < 10; ++round) {
    if (round > 0) { /* the key is bumped by the Weyl constants between rounds */
      k0 += W0;
      k1 += W1;
    }
    uint64_t p0 = (uint64_t)M0 * (uint64_t)c0;
    uint64_t p1 = (uint64_t)M1 * (uint64_t)c2;
    uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
    uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
    uint32_t n0 = hi1 ^ c1 ^ k0;
    uint32_t n1 = lo1;
    uint32_t n2 = hi0 ^ c3 ^ k1;
    uint32_t n3 = lo0;
    c0 = n0; c1 = n1; c2 = n2; c3 = n3;
  }
  out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

/* Random word feeding dimension m of sample s in iteration `iter`:
 * counter = (s lo32, s hi32, iter, m / 4), key = (seed, task key),
 * word = output[m % 4]. */
static uint32_t sample_word(uint32_t seed, uint32_t task_key, uint32_t iter,
                            uint64_t s, int m) {
  uint32_t ctr[4] = {(uint32_t)s, (uint32_t)(s >> 32), iter, (uint32_t)(m / 4)};
  uint32_t key[2] = {seed, task_key};
  uint32_t out[4];
  orc_philox4x32_10(ctr, key, out);
  return out[m % 4];
}

/* ------------------------------------------------------------------------ */
/* Diagrams                                                                  */
/* ------------------------------------------------------------------------ */

typedef struct {
  int order;
  int id;
  int M[ORC_MAXN][ORC_MAXN];
  int nlines, nloops, ncuts, ndim;
  int tail[ORC_MAXLINES], head[ORC_MAXLINES];
  int is_particle[ORC_MAXLINES];
  int vout[ORC_MAXN][2], vin[ORC_MAXN][2]; /* <o1 o2|V|i1 i2> line ids */
  int loop_line[ORC_MAXLOOPS];             /* line carrying loop momentum l */
  int coef[ORC_MAXLINES][ORC_MAXLOOPS];    /* k_line = sum coef * k_loop */
  int cut[ORC_MAXCUTS][ORC_MAXLINES];      /* +1 hole crosses, -1 particle */
  int n_eq, n_h, n_cycles;
  double prefactor;
} orc_diagram;

/* All matrices of one order in lexicographic order of their row-major digits. */
typedef struct {
  int count;
  int (*mats)[ORC_MAXN * ORC_MAXN];
} orc_diag_list;

static orc_diag_list g_lists[ORC_MAXN + 1];

static int connected(int n, int M[ORC_MAXN][ORC_MAXN]) {
  int seen[ORC_MAXN] = {0};
  int stack[ORC_MAXN], sp = 0;
  seen[0] = 1;
  stack[sp++] = 0;
  while (sp) {
    int u = stack[--sp];
    for (int v = 0; v < n; ++v)
      if (!seen[v] && (M[u][v] + M[v][u]) > 0) {
        seen[v] = 1;
        stack[sp++] = v;
      }
  }
  for (int v = 0; v < n; ++v)
    if (!seen[v]) return 0;
  return 1;
}

/* Candidate rows for row u: digit vectors over {0,1,2} with zero at u and
 * digit sum 2, listed in increasing lexicographic order. */
static int row_candidates(int n, int u, int rows[][ORC_MAXN]) {
  int cnt = 0;
  int total = 1;
  for (int i = 0; i < n; ++i) total *= 3;
  for (int code = 0; code < total; ++code) {
    int digits[ORC_MAXN];
    int c = code, sum = 0;
    for (int i = n - 1; i >= 0; --i) { /* most significant digit first */
      digits[i] = c % 3;
      c /= 3;
    }
    for (int i = 0; i < n; ++i) sum += digits[i];
    if (sum != 2 || digits[u] != 0) continue;
    memcpy(rows[cnt], digits, sizeof(int) * n);
    ++cnt;
  }
  return cnt;
}

static void build_list(int n) {
  if (g_lists[n].mats) return;
  if (n == 1) {
    g_lists[1].count = 1;
    g_lists[1].mats = calloc(1, sizeof(*g_lists[1].mats));
    g_lists[1].mats[0][0] = 2; /* the first-order diagram: one vertex, two hole self-lines */
    return;
  }
  int rows[ORC_MAXN][64][ORC_MAXN];
  int nrows[ORC_MAXN];
  for (int u = 0; u < n; ++u) nrows[u] = row_candidates(n, u, rows[u]);
  int cap = 1024, count = 0;
  int (*mats)[ORC_MAXN * ORC_MAXN] = malloc(sizeof(*mats) * cap);
  int idx[ORC_MAXN] = {0};
  for (;;) {
    int M[ORC_MAXN][ORC_MAXN] = {{0}};
    for (int u = 0; u < n; ++u)
      for (int v = 0; v < n; ++v) M[u][v] = rows[u][idx[u]][v];
    int ok = 1;
    for (int v = 0; v < n && ok; ++v) {
      int cs = 0;
      for (int u = 0; u < n; ++u) cs += M[u][v];
      if (cs != 2) ok = 0;
    }
    if (ok && connected(n, M)) {
      if (count == cap) {
        cap *= 2;
        mats = realloc(mats, sizeof(*mats) * cap);
      }
      memset(mats[count], 0, sizeof(mats[count]));
      for (int u = 0; u < n; ++u)
        for (int v = 0; v < n; ++v) mats[count][u * ORC_MAXN + v] = M[u][v];
      ++count;
    }
    /* odometer, last row fastest: lexicographic order of the flattened matrix */
    int r = n - 1;
    while (r >= 0) {
      if (++idx[r] < nrows[r]) break;
      idx[r] = 0;
      --r;
    }
    if (r < 0) break;
  }
  g_lists[n].count = count;
  g_lists[n].mats = mats;
}

int orc_num_diagrams(int order) {
  if (order < 1 || order > ORC_MAXN) return -1;
  build_list(order);
  return g_lists[order].count;
}

/* Solve A X = B (n x n, nrhs columns) by Gaussian elimination with partial
 * pivoting; A and B are overwritten.  Returns 0 on success. */
static int gauss_solve(int n, int nrhs, double A[][ORC_MAXLINES],
                       double B[][ORC_MAXLOOPS]) {
  for (int col = 0; col < n; ++col) {
    int piv = col;
    for (int r = col + 1; r < n; ++r)
      if (fabs(A[r][col]) > fabs(A[piv][col])) piv = r;
    if (fabs(A[piv][col]) < 1e-12) return -1;
    if (piv != col) {
      for (int c = 0; c < n; ++c) {
        double t = A[col][c]; A[col][c] = A[piv][c]; A[piv][c] = t;
      }
      for (int c = 0; c < nrhs; ++c) {
        double t = B[col][c]; B[col][c] = B[piv][c]; B[piv][c] = t;
      }
    }
    for (int r = 0; r < n; ++r) {
      if (r == col) continue;
      double f = A[r][col] / A[col][col];
      if (f == 0.0) continue;
      for (int c = 0; c < n; ++c) A[r][c] -= f * A[col][c];
      for (int c = 0; c < nrhs; ++c) B[r][c] -= f * B[col][c];
    }
  }
  for (int r = 0; r < n; ++r)
    for (int c = 0; c < nrhs; ++c) B[r][c] /= A[r][r];
  return 0;
}

static int uf_find(int *p, int x) {
  while (p[x] != x) x = p[x];
  return x;
}

/* Build one diagram: lines, vertex slots, loop momenta, routing, cuts and
 * prefactor.  Returns 0 on success. */
int orc_get_diagram(int order, int id, orc_diagram *d) {
  if (order < 1 || order > ORC_MAXN) return -1;
  build_list(order);
  if (id < 0 || id >= g_lists[order].count) return -1;
  memset(d, 0, sizeof(*d));
  int n = order;
  d->order = n;
  d->id = id;
  for (int u = 0; u < n; ++u)
    for (int v = 0; v < n; ++v) d->M[u][v] = g_lists[order].mats[id][u * ORC_MAXN + v];

  /* Lines: particle lines (u < v) first, in lexicographic (u, v) order, then
   * hole lines (u > v, and the first-order self-lines) in lexicographic order. */
  int nl = 0;
  for (int u = 0; u < n; ++u)
    for (int v = u + 1; v < n; ++v)
      for (int c = 0; c < d->M[u][v]; ++c) {
        d->tail[nl] = u; d->head[nl] = v; d->is_particle[nl] = 1; ++nl;
      }
  for (int u = 0; u < n; ++u)
    for (int v = 0; v <= u; ++v) {
      if (v == u && n > 1) continue;
      for (int c = 0; c < d->M[u][v]; ++c) {
        d->tail[nl] = u; d->head[nl] = v; d->is_particle[nl] = 0; ++nl;
      }
    }
  d->nlines = nl;
  d->nloops = n + 1;
  d->ncuts = n - 1;
  d->ndim = 3 * d->nloops;

  /* Vertex slots: out lines (leaving the vertex) and in lines (entering it),
   * each sorted by line index; the matrix element is <o1 o2|V|i1 i2>. */
  for (int v = 0; v < n; ++v) {
    int no = 0, ni = 0;
    for (int l = 0; l < nl; ++l) {
      if (d->tail[l] == v) d->vout[v][no++] = l;
      if (d->head[l] == v) d->vin[v][ni++] = l;
    }
    if (no != 2 || ni != 2) return -2;
  }

  /* n_h, n_eq, closed loops of the reference pairing (o1<->i1, o2<->i2). */
  d->n_h = 0;
  for (int l = 0; l < nl; ++l) d->n_h += !d->is_particle[l];
  d->n_eq = (n == 1) ? 1 : 0;
  for (int u = 0; u < n; ++u)
    for (int v = 0; v < n; ++v)
      if (u != v && d->M[u][v] == 2) d->n_eq++;
  {
    int succ[ORC_MAXLINES];
    for (int l = 0; l < nl; ++l) {
      int v = d->head[l];
      int slot = (d->vin[v][0] == l) ? 0 : 1;
      succ[l] = d->vout[v][slot];
    }
    int seen[ORC_MAXLINES] = {0};
    d->n_cycles = 0;
    for (int l = 0; l < nl; ++l) {
      if (seen[l]) continue;
      d->n_cycles++;
      int x = l;
      while (!seen[x]) { seen[x] = 1; x = succ[x]; }
    }
  }
  d->prefactor = pow(0.5, d->n_eq) * (((d->n_h + d->n_cycles) % 2) ? -1.0 : 1.0);

  /* Loop momenta: lines taken greedily in index order into a spanning forest
   * (union-find); lines that would close a cycle carry the loop momenta, in
   * index order. */
  {
    int parent[ORC_MAXN];
    for (int v = 0; v < n; ++v) parent[v] = v;
    int nloop = 0;
    for (int l = 0; l < nl; ++l) {
      int a = uf_find(parent, d->tail[l]), b = uf_find(parent, d->head[l]);
      if (a != b) parent[a] = b;
      else {
        if (nloop >= ORC_MAXLOOPS) return -3;
        d->loop_line[nloop++] = l;
      }
    }
    if (nloop != d->nloops) return -3;
  }

  /* Routing: solve the linear system {k_loopline(l) = e_l ; momentum in =
   * momentum out at vertices 1..n-1} for the line momenta. */
  {
    double A[ORC_MAXLINES][ORC_MAXLINES];
    double B[ORC_MAXLINES][ORC_MAXLOOPS];
    memset(A, 0, sizeof(A));
    memset(B, 0, sizeof(B));
    int row = 0;
    for (int l = 0; l < d->nloops; ++l) {
      A[row][d->loop_line[l]] = 1.0;
      B[row][l] = 1.0;
      ++row;
    }
    for (int v = 1; v < n; ++v) {
      for (int l = 0; l < nl; ++l) {
        if (d->head[l] == v) A[row][l] += 1.0;
        if (d->tail[l] == v) A[row][l] -= 1.0;
      }
      ++row;
    }
    if (row != nl) return -4;
    if (gauss_solve(nl, d->nloops, A, B)) return -4;
    for (int l = 0; l < nl; ++l)
      for (int k = 0; k < d->nloops; ++k) {
        double c = B[l][k];
        double r = floor(c + 0.5);
        if (fabs(c - r) > 1e-9) return -5;
        d->coef[l][k] = (int)r;
      }
  }

  /* Cuts between time levels c and c+1. */
  for (int c = 0; c < d->ncuts; ++c)
    for (int l = 0; l < nl; ++l) {
      int lo = d->tail[l] < d->head[l] ? d->tail[l] : d->head[l];
      int hi = d->tail[l] < d->head[l] ? d->head[l] : d->tail[l];
      d->cut[c][l] = (lo <= c && c < hi) ? (d->is_particle[l] ? -1 : +1) : 0;
    }
  return 0;
}

/* ------------------------------------------------------------------------ */
/* Problem and integrand                                                     */
/* ------------------------------------------------------------------------ */

typedef struct {
  int order, diagram_id;
  int q;                  /* 2: neutron matter (spin labels); 4: spin x isospin */
  double density;         /* total nucleon density n [fm^-3] */
  double proton_fraction; /* x = n_p / n */
  double C0;              /* [fm^2] */
  double Cy;              /* [dimensionless]: Cy/(q^2 + mpi^2) in fm^2 */
  double mpi, Lambda;     /* [fm^-1] */
  double reg_exp;         /* regulator exponent */
  double hbar2_m;         /* hbar^2/m [MeV fm^2] */
  double hbarc;           /* [MeV fm] */
  int n_bins;
  double alpha;
  double kcut_extra;      /* particle-loop radius = kF,max + kcut_extra * Lambda */
  uint32_t seed, task_key;
  int label_method;       /* 0: brute force over q^{2n}; 1: closed-loop rule */
  int spectrum;           /* 0: free eps = hbar^2 k^2 / 2m; 1: Hartree-Fock (eq:spe) */
  int hf_n;               /* HF: spline intervals on [0, hf_kmax] */
  double hf_kmax;         /* HF: table range; Sigma = its last node value beyond */
  const double *hf_y;     /* HF: Sigma_tau(k_i), tau = n then p, 2 x (hf_n + 1) */
  const double *hf_m;     /* HF: spline second derivatives, same layout */
  int group;              /* -1: diagram_id alone; p >= 0: the group of the order's
                             diagrams with p particle-carried loops (diagram_id unused) */
  int reg_k;              /* regularised components k = 1..reg_k (at most ORC_MAXREG) */
  double reg_eta;         /* component k replaces every D_c by D_c - k reg_eta [MeV] */
  int train_iters;        /* > 0: training/evaluation phases (Sec. "MC integration"):
                             the first train_iters iterations adapt the grid, the rest
                             keep it frozen and alone make the combined estimate */
} orc_problem;

typedef struct {
  double kF[2];   /* neutron, proton Fermi momenta */
  double kFmax;
  double Rhole, Rpart;
} orc_medium;

static void medium_of(const orc_problem *pb, orc_medium *md) {
  double x = pb->proton_fraction;
  double nn = (1.0 - x) * pb->density, np = x * pb->density;
  md->kF[0] = cbrt(3.0 * M_PI * M_PI * nn);
  md->kF[1] = cbrt(3.0 * M_PI * M_PI * np);
  md->kFmax = md->kF[0] > md->kF[1] ? md->kF[0] : md->kF[1];
  md->Rhole = md->kFmax;
  md->Rpart = md->kFmax + pb->kcut_extra * pb->Lambda;
}

/* V(p, p') [MeV fm^3] for 3-vectors p, p' (relative momenta). */
static double pot(const orc_problem *pb, const double p[3], const double pp[3]) {
  double q2 = 0, p2 = 0, pp2 = 0;
  for (int i = 0; i < 3; ++i) {
    double qi = p[i] - pp[i];
    q2 += qi * qi;
    p2 += p[i] * p[i];
    pp2 += pp[i] * pp[i];
  }
  double fp = exp(-pow(sqrt(p2) / pb->Lambda, pb->reg_exp));
  double fpp = exp(-pow(sqrt(pp2) / pb->Lambda, pb->reg_exp));
  return pb->hbarc * (pb->C0 + pb->Cy / (q2 + pb->mpi * pb->mpi)) * fp * fpp;
}

/* ------------------------------------------------------------------------ */
/* Hartree-Fock single-particle energies (eq:spe)                            */
/* ------------------------------------------------------------------------ */

/* Gauss-Legendre rule on [-1, 1]: nodes are the roots of P_n (Newton from
 * the usual cosine guesses), weights 2 / ((1 - x^2) P_n'(x)^2). */
void orc_gauss_legendre(int n, double *x, double *w) {
  for (int i = 0; i < (n + 1) / 2; ++i) {
    double z = cos(M_PI * (i + 0.75) / (n + 0.5)), dp = 1.0;
    for (int it = 0; it < 200; ++it) {
      double p1 = 1.0, p0 = 0.0;
      for (int j = 1; j <= n; ++j) {
        const double pm = p0;
        p0 = p1;
        p1 = ((2.0 * j - 1.0) * z * p0 - (j - 1.0) * pm) / j;
      }
      dp = n * (z * p1 - p0) / (z * z - 1.0);
      const double dz = p1 / dp;
      z -= dz;
      if (fabs(dz) < 1e-17) break;
    }
    x[i] = -z;
    x[n - 1 - i] = z;
    w[i] = w[n - 1 - i] = 2.0 / ((1.0 - z * z) * dp * dp);
  }
}

/* HF self-energy Sigma_tau(k) [MeV] of a nucleon of isospin tau (0 n, 1 p):
 * the sum over occupied partners j of <ij|Vbar|ij>, Vbar = V (1 - P12).  With
 * p = (k - k') / 2 the direct element is V(p, p) for every partner spin (2
 * spins) and the exchange element V(p, -p) needs equal spin and isospin:
 *   Sigma_tau(k) = sum_tau' \int_{k' < kF_tau'} d^3k' / (2 pi)^3
 *                  [2 V(p, p) - delta_{tau tau'} V(p, -p)].
 * Neutron matter (q = 2) has only tau' = n.  ng-point Gauss-Legendre in |k'|
 * and in the cosine of the angle between k and k'. */
double orc_hf_sigma(const orc_problem *pb, int tau, double k, int ng) {
  double xg[256], wg[256];
  if (ng > 256) ng = 256;
  orc_gauss_legendre(ng, xg, wg);
  const double x = pb->q == 4 ? pb->proton_fraction : 0.0;
  const double kF[2] = {cbrt(3.0 * M_PI * M_PI * (1.0 - x) * pb->density),
                        cbrt(3.0 * M_PI * M_PI * x * pb->density)};
  double total = 0.0;
  for (int tp = 0; tp < (pb->q == 4 ? 2 : 1); ++tp) {
    if (kF[tp] <= 0.0) continue;
    double sum = 0.0;
    for (int a = 0; a < ng; ++a) {
      const double kp = 0.5 * kF[tp] * (xg[a] + 1.0), wk = 0.5 * kF[tp] * wg[a];
      for (int b = 0; b < ng; ++b) {
        const double mu = xg[b], sn = sqrt(fmax(0.0, 1.0 - mu * mu));
        double p[3] = {-0.5 * kp * sn, 0.0, 0.5 * (k - kp * mu)};
        double mp[3] = {-p[0], -p[1], -p[2]};
        double f = 2.0 * pot(pb, p, p);
        if (tp == tau) f -= pot(pb, p, mp);
        sum += wk * wg[b] * kp * kp * f;
      }
    }
    total += sum * 2.0 * M_PI / pow(2.0 * M_PI, 3.0);
  }
  return total;
}

/* Cubic spline through y_0..y_n at spacing h with zero end slopes (Sigma is
 * even in k, and flat where the regulator has switched it off): second
 * derivatives m from
 *   2 m_0 + m_1 = 6 (y_1 - y_0) / h^2,
 *   m_{i-1} + 4 m_i + m_{i+1} = 6 (y_{i+1} - 2 y_i + y_{i-1}) / h^2,
 *   m_{n-1} + 2 m_n = -6 (y_n - y_{n-1}) / h^2,
 * solved by the Thomas algorithm. */
void orc_spline_flat_ends(int n, double h, const double *y, double *m) {
  static double a[4097], b[4097], c[4097], r[4097];
  if (n < 2 || n > 4096) return;
  for (int i = 0; i <= n; ++i) {
    a[i] = 1.0;
    b[i] = 4.0;
    c[i] = 1.0;
  }
  b[0] = b[n] = 2.0;
  r[0] = 6.0 * (y[1] - y[0]) / (h * h);
  for (int i = 1; i < n; ++i) r[i] = 6.0 * (y[i + 1] - 2.0 * y[i] + y[i - 1]) / (h * h);
  r[n] = -6.0 * (y[n] - y[n - 1]) / (h * h);
  /* forward elimination */
  for (int i = 1; i <= n; ++i) {
    const double f = a[i] / b[i - 1];
    b[i] -= f * c[i - 1];
    r[i] -= f * r[i - 1];
  }
  m[n] = r[n] / b[n];
  for (int i = n - 1; i >= 0; --i) m[i] = (r[i] - c[i] * m[i + 1]) / b[i];
}

/* The spline at k (constant beyond the last node). */
static double spline_eval(int n, double h, const double *y, const double *m, double k) {
  if (k >= n * h) return y[n];
  int i = (int)(k / h);
  if (i > n - 1) i = n - 1;
  const double t = (k - i * h) / h, u = 1.0 - t;
  return u * y[i] + t * y[i + 1] + h * h / 6.0 * ((u * u * u - u) * m[i] + (t * t * t - t) * m[i + 1]);
}

double orc_hf_spline_eval(const orc_problem *pb, int tau, double k) {
  const double h = pb->hf_kmax / pb->hf_n;
  const int off = tau * (pb->hf_n + 1);
  return spline_eval(pb->hf_n, h, pb->hf_y + off, pb->hf_m + off, k);
}

/* Integrand in loop-momentum space, as a contribution to E/N [MeV]:
 *   f = prefactor * (2pi)^{-3L} * [sum over labels of Pauli * prod <..|Vbar|..>]
 *       / prod_c D_c / n.
 * Also returns the condition scale (same expression with every label term
 * and every denominator taken in absolute value, times 1 + sum of the
 * denominator and regulator condition numbers) and the largest |D| condition
 * number seen. */
#define ORC_MAXREG 4

typedef struct {
  double f;
  double freg[ORC_MAXREG];  /* regularised components k = 1..reg_k */
  double wcond;   /* condition scale, positive */
  double labelsum;
  double labelabs;
  int pauli_any;  /* 0 if every label assignment is Pauli-blocked */
} orc_point;

static int tau_of(int q, int label) { return q == 4 ? (label >> 1) : 0; }

static void eval_point(const orc_problem *pb, const orc_diagram *d,
                       const orc_medium *md, const double kl[][3],
                       orc_point *out) {
  const int n = d->order, nl = d->nlines, L = d->nloops;
  double k[ORC_MAXLINES][3], k2[ORC_MAXLINES], eps[ORC_MAXLINES];
  double epst[ORC_MAXLINES][2];  /* per isospin (HF spectrum) */
  for (int l = 0; l < nl; ++l) {
    for (int i = 0; i < 3; ++i) {
      double s = 0;
      for (int j = 0; j < L; ++j) s += d->coef[l][j] * kl[j][i];
      k[l][i] = s;
    }
    k2[l] = k[l][0] * k[l][0] + k[l][1] * k[l][1] + k[l][2] * k[l][2];
    eps[l] = 0.5 * pb->hbar2_m * k2[l];
    for (int t = 0; t < 2; ++t)
      epst[l][t] = eps[l] + (pb->spectrum ? orc_hf_spline_eval(pb, t, sqrt(k2[l])) : 0.0);
    eps[l] = epst[l][0];
  }
  /* HF energies of nuclear matter depend on each line's isospin: the
   * denominators are then taken per label assignment (brute force only) */
  const int iso_den = pb->spectrum && pb->q == 4;
  if (iso_den && pb->label_method != 0) {
    out->f = NAN;
    out->wcond = NAN;
    out->labelsum = out->labelabs = NAN;
    out->pauli_any = 1;
    return;
  }
  /* occupation factors per line and isospin: n_k for holes, 1 - n_k for particles */
  double P[ORC_MAXLINES][2];
  for (int l = 0; l < nl; ++l)
    for (int t = 0; t < 2; ++t) {
      double occ = (k2[l] < md->kF[t] * md->kF[t]) ? 1.0 : 0.0;
      P[l][t] = d->is_particle[l] ? 1.0 - occ : occ;
    }
  /* matrix elements per vertex: direct V(p, p') and exchange V(p, -p') */
  double Vd[ORC_MAXN], Ve[ORC_MAXN], regcond = 0.0;
  for (int v = 0; v < n; ++v) {
    double p[3], pp[3], mpp[3];
    for (int i = 0; i < 3; ++i) {
      p[i] = 0.5 * (k[d->vout[v][0]][i] - k[d->vout[v][1]][i]);
      pp[i] = 0.5 * (k[d->vin[v][0]][i] - k[d->vin[v][1]][i]);
      mpp[i] = -pp[i];
    }
    Vd[v] = pot(pb, p, pp);
    Ve[v] = pot(pb, p, mpp);
    double pn = sqrt(p[0] * p[0] + p[1] * p[1] + p[2] * p[2]);
    double ppn = sqrt(pp[0] * pp[0] + pp[1] * pp[1] + pp[2] * pp[2]);
    regcond += pb->reg_exp * (pow(pn / pb->Lambda, pb->reg_exp) +
                              pow(ppn / pb->Lambda, pb->reg_exp));
  }
  /* spin(-isospin) sum */
  const int q = pb->q;
  double ls = 0.0, lsabs = 0.0;
  int any = 0;
  if (pb->label_method == 0) {
    long total = 1;
    for (int l = 0; l < nl; ++l) total *= q;
    for (long code = 0; code < total; ++code) {
      int lab[ORC_MAXLINES];
      long c = code;
      for (int l = 0; l < nl; ++l) { lab[l] = (int)(c % q); c /= q; }
      double pauli = 1.0;
      for (int l = 0; l < nl; ++l) pauli *= P[l][tau_of(q, lab[l])];
      if (pauli == 0.0) continue;
      double prod = 1.0, prodabs = 1.0;
      for (int v = 0; v < n; ++v) {
        int o1 = lab[d->vout[v][0]], o2 = lab[d->vout[v][1]];
        int i1 = lab[d->vin[v][0]], i2 = lab[d->vin[v][1]];
        double dir = (o1 == i1 && o2 == i2) ? 1.0 : 0.0;
        double exc = (o1 == i2 && o2 == i1) ? 1.0 : 0.0;
        prod *= dir * Vd[v] - exc * Ve[v];
        prodabs *= dir * fabs(Vd[v]) + exc * fabs(Ve[v]);
      }
      if (prodabs != 0.0) any = 1;
      if (iso_den && prodabs != 0.0) {
        double dp = 1.0, dc = 0.0;
        for (int c = 0; c < d->ncuts; ++c) {
          double D = 0.0, Dabs = 0.0;
          for (int l = 0; l < nl; ++l) {
            const double e = epst[l][tau_of(q, lab[l])];
            D += d->cut[c][l] * e;
            Dabs += d->cut[c][l] ? fabs(e) : 0.0;
          }
          dp *= D;
          dc += Dabs / fabs(D);
        }
        ls += pauli * prod / dp;
        lsabs += pauli * prodabs / fabs(dp) * (1.0 + dc + regcond);
        continue;
      }
      ls += pauli * prod;
      lsabs += pauli * prodabs;
    }
  } else {
    /* closed-loop rule: expand every vertex into direct / exchange; the label
     * deltas then force one label per cycle of the resulting line permutation,
     * and each cycle contributes sum_{labels} prod_{lines in cycle} Pauli. */
    for (int E = 0; E < (1 << n); ++E) {
      double coef = 1.0, coefabs = 1.0;
      int succ[ORC_MAXLINES];
      for (int v = 0; v < n; ++v) {
        int ex = (E >> v) & 1;
        coef *= ex ? -Ve[v] : Vd[v];
        coefabs *= ex ? fabs(Ve[v]) : fabs(Vd[v]);
      }
      for (int l = 0; l < nl; ++l) {
        int v = d->head[l];
        int slot = (d->vin[v][0] == l) ? 0 : 1;
        if ((E >> v) & 1) slot = 1 - slot;
        succ[l] = d->vout[v][slot];
      }
      int seen[ORC_MAXLINES] = {0};
      double trace = 1.0;
      for (int l = 0; l < nl && trace != 0.0; ++l) {
        if (seen[l]) continue;
        double tsum = 0.0;
        for (int lab = 0; lab < q; ++lab) {
          double prod = 1.0;
          int x = l;
          do {
            prod *= P[x][tau_of(q, lab)];
            x = succ[x];
          } while (x != l);
          tsum += prod;
        }
        int x = l;
        do { seen[x] = 1; x = succ[x]; } while (x != l);
        trace *= tsum;
      }
      if (trace != 0.0 && coefabs != 0.0) any = 1;
      ls += coef * trace;
      lsabs += coefabs * trace;
    }
  }
  /* denominators */
  double dprod = 1.0, dcond = 0.0;
  for (int c = 0; c < d->ncuts; ++c) {
    double D = 0.0, Dabs = 0.0;
    for (int l = 0; l < nl; ++l) {
      D += d->cut[c][l] * eps[l];
      Dabs += d->cut[c][l] ? fabs(eps[l]) : 0.0;
    }
    dprod *= D;
    if (any) dcond += Dabs / fabs(D);
  }
  double measure = pow(2.0 * M_PI, -3.0 * L);
  out->labelsum = ls;
  out->labelabs = lsabs;
  out->pauli_any = any;
  for (int k = 0; k < ORC_MAXREG; ++k) out->freg[k] = 0.0;
  if (!any) {
    out->f = 0.0;
    out->wcond = 0.0;
    return;
  }
  if (pb->reg_k > 0) {
    /* regularised denominators D_c - eta_k (D_c < 0 for every allowed
     * configuration of a Goldstone diagram: the shift moves the pole away) */
    if (iso_den) {
      for (int k = 0; k < pb->reg_k; ++k) out->freg[k] = NAN;
    } else {
      for (int k = 0; k < pb->reg_k; ++k) {
        const double eta = (k + 1) * pb->reg_eta;
        double dk = 1.0;
        for (int c = 0; c < d->ncuts; ++c) {
          double D = 0.0;
          for (int l = 0; l < nl; ++l) D += d->cut[c][l] * eps[l];
          dk *= D - eta;
        }
        out->freg[k] = d->prefactor * measure / pb->density / dk * ls;
      }
    }
  }
  if (iso_den) {
    /* denominators already inside ls; lsabs carries the condition terms */
    const double sc = d->prefactor * measure / pb->density;
    out->f = sc * ls;
    out->wcond = fabs(sc) * lsabs;
    return;
  }
  double scale = d->prefactor * measure / pb->density / dprod;
  out->f = scale * ls;
  out->wcond = fabs(scale) * lsabs * (1.0 + dcond + regcond);
}

/* ------------------------------------------------------------------------ */
/* Hypercube -> loop momenta through the VEGAS map                          */
/* ------------------------------------------------------------------------ */

/* VEGAS map of one sample (uniform -> bin, fraction -> x): for dimension m the
 * Philox word w gives bin b = floor(w N_b / 2^32) and fraction
 * r = ((w N_b mod 2^32) + 1/2) / 2^32, then x = e_b + r (e_{b+1} - e_b) and the
 * Jacobian picks up N_b (e_{b+1} - e_b).  Returns the Jacobian. */
static double vegas_map(int nd, int nb, const double *edges, uint32_t seed,
                        uint32_t task_key, uint32_t iter, uint64_t s, double *x,
                        int *bins) {
  double jac = 1.0;
  for (int m = 0; m < nd; ++m) {
    uint32_t w = sample_word(seed, task_key, iter, s, m);
    uint64_t wn = (uint64_t)w * (uint64_t)nb;
    int b = (int)(wn >> 32);
    uint32_t lo = (uint32_t)wn;
    double r = ((double)lo + 0.5) * 0x1p-32;
    const double *e = edges + (size_t)m * (nb + 1);
    double width = e[b + 1] - e[b];
    x[m] = e[b] + r * width;
    jac *= nb * width;
    bins[m] = b;
  }
  return jac;
}

/* Unit hypercube -> loop momenta, loop-major (radius, cos theta, azimuth):
 * radius = R x0, cos theta = 2 x1 - 1, azimuth = 2 pi x2, Jacobian
 * R radius^2 * 2 * 2 pi per loop.  R = kF,max for loops carried by a hole line
 * (exact bound) and kF,max + kcut_extra * Lambda for particle lines
 * (truncation; the regulators make the cut-off tail negligible). */
static double loop_momenta(const orc_diagram *d, const orc_medium *md,
                           const double *x, double kl[][3]) {
  double jac = 1.0;
  for (int l = 0; l < d->nloops; ++l) {
    double R = d->is_particle[d->loop_line[l]] ? md->Rpart : md->Rhole;
    double rad = R * x[3 * l];
    double ct = 2.0 * x[3 * l + 1] - 1.0;
    double st = sqrt(fmax(0.0, (1.0 - ct) * (1.0 + ct)));
    double ph = 2.0 * M_PI * x[3 * l + 2];
    kl[l][0] = rad * st * cos(ph);
    kl[l][1] = rad * st * sin(ph);
    kl[l][2] = rad * ct;
    jac *= R * rad * rad * 2.0 * (2.0 * M_PI);
  }
  return jac;
}

/* Physics integrand in the unit hypercube: w(x) = J_sphere * f(k(x)). */
typedef struct {
  const orc_problem *pb;
  const orc_diagram *d;
  const orc_medium *md;
} phys_ctx;

static double phys_eval(const void *ctx, const double *x, double *wcond, double *wreg) {
  const phys_ctx *c = (const phys_ctx *)ctx;
  double kl[ORC_MAXLOOPS][3];
  double jac = loop_momenta(c->d, c->md, x, kl);
  orc_point pt;
  eval_point(c->pb, c->d, c->md, (const double(*)[3])kl, &pt);
  if (wcond) *wcond = fabs(jac) * pt.wcond;
  if (wreg)
    for (int k = 0; k < c->pb->reg_k; ++k) wreg[k] = jac * pt.freg[k];
  return jac * pt.f;
}

/* ------------------------------------------------------------------------ */
/* Diagram groups                                                            */
/* ------------------------------------------------------------------------ */

/* Particle-carried loops of a diagram: the loop momenta whose carrying line
 * is a particle line.  With the spanning forest built particle lines first
 * this is the cycle rank of the particle-line subgraph, a property of the
 * diagram; grouping by it is this implementation's reading of the paper's
 * grouping by particle-hole composition (it gives 1, 2, 4, 5 groups at orders
 * 2..5, as Table I's N_grp). */
static int particle_loops(const orc_diagram *d) {
  int p = 0;
  for (int j = 0; j < d->nloops; ++j) p += d->is_particle[d->loop_line[j]] ? 1 : 0;
  return p;
}

/* Ids of the diagrams of `order` with p particle-carried loops, ascending;
 * returns their number (ids written up to cap). */
int orc_group_members(int order, int p, int *ids, int cap) {
  int n = 0, nd = orc_num_diagrams(order);
  for (int i = 0; i < nd; ++i) {
    orc_diagram d;
    if (orc_get_diagram(order, i, &d)) return -1;
    if (particle_loops(&d) != p) continue;
    if (ids && n < cap) ids[n] = i;
    ++n;
  }
  return n;
}

/* A group's integrand at hypercube point x: the members' integrands summed,
 * each member's loop momenta taken in the canonical order -- its particle
 * loops first, then its hole loops, each in its own order -- so that loop c
 * has the radius of a particle loop for c < p and of a hole loop otherwise. */
typedef struct {
  const orc_problem *pb;
  const orc_medium *md;
  int n, p, L;
  orc_diagram *d;            /* n members */
  int (*canon)[ORC_MAXLOOPS]; /* canon[i][c] = member i's loop at canonical slot c */
} group_ctx;

static double group_eval(const void *ctx, const double *x, double *wcond, double *wreg) {
  const group_ctx *g = (const group_ctx *)ctx;
  double kc[ORC_MAXLOOPS][3], jac = 1.0;
  for (int c = 0; c < g->L; ++c) {
    double R = c < g->p ? g->md->Rpart : g->md->Rhole;
    double rad = R * x[3 * c];
    double ct = 2.0 * x[3 * c + 1] - 1.0;
    double st = sqrt(fmax(0.0, (1.0 - ct) * (1.0 + ct)));
    double ph = 2.0 * M_PI * x[3 * c + 2];
    kc[c][0] = rad * st * cos(ph);
    kc[c][1] = rad * st * sin(ph);
    kc[c][2] = rad * ct;
    jac *= R * rad * rad * 2.0 * (2.0 * M_PI);
  }
  double f = 0.0, wc = 0.0, fr[ORC_MAXREG] = {0.0, 0.0, 0.0, 0.0};
  for (int i = 0; i < g->n; ++i) {
    double kl[ORC_MAXLOOPS][3];
    for (int c = 0; c < g->L; ++c)
      for (int a = 0; a < 3; ++a) kl[g->canon[i][c]][a] = kc[c][a];
    orc_point pt;
    eval_point(g->pb, &g->d[i], g->md, (const double(*)[3])kl, &pt);
    f += pt.f;
    wc += pt.wcond;
    for (int k = 0; k < g->pb->reg_k; ++k) fr[k] += pt.freg[k];
  }
  if (wcond) *wcond = fabs(jac) * wc;
  if (wreg)
    for (int k = 0; k < g->pb->reg_k; ++k) wreg[k] = jac * fr[k];
  return jac * f;
}

/* Members and canonical loop orders of pb's group; returns 0 or < 0. */
static int group_setup(const orc_problem *pb, const orc_medium *md, group_ctx *g) {
  g->pb = pb;
  g->md = md;
  g->p = pb->group;
  g->L = pb->order + 1;
  g->n = orc_group_members(pb->order, pb->group, NULL, 0);
  if (g->n <= 0) return -1;
  g->d = (orc_diagram *)malloc(sizeof(orc_diagram) * g->n);
  g->canon = malloc(sizeof(*g->canon) * g->n);
  int *ids = (int *)malloc(sizeof(int) * g->n);
  orc_group_members(pb->order, pb->group, ids, g->n);
  for (int i = 0; i < g->n; ++i) {
    orc_get_diagram(pb->order, ids[i], &g->d[i]);
    int c = 0;
    for (int pass = 0; pass < 2; ++pass)
      for (int j = 0; j < g->L; ++j) {
        const int part = g->d[i].is_particle[g->d[i].loop_line[j]] ? 1 : 0;
        if ((pass == 0) == (part == 1)) g->canon[i][c++] = j;
      }
  }
  free(ids);
  return 0;
}

static void group_free(group_ctx *g) {
  free(g->d);
  free(g->canon);
}

/* Separable test integrand prod_m g(x_m), g a normalised Gaussian of width
 * `width` centred at 1/2 restricted to [0, 1]; its integral is
 * erf(1/(2 sqrt(2) width))^nd. */
typedef struct {
  double width;
  int nd;
} gauss_ctx;

static double gauss_eval(const void *ctx, const double *x, double *wcond, double *wreg) {
  (void)wreg;
  const gauss_ctx *g = (const gauss_ctx *)ctx;
  double v = 1.0;
  for (int m = 0; m < g->nd; ++m) {
    double t = (x[m] - 0.5) / g->width;
    v *= exp(-0.5 * t * t) / (g->width * sqrt(2.0 * M_PI));
  }
  if (wcond) *wcond = fabs(v);
  return v;
}

typedef double (*integrand_fn)(const void *ctx, const double *x, double *wcond,
                               double *wreg);

/* ------------------------------------------------------------------------ */
/* Exported evaluation entry points                                          */
/* ------------------------------------------------------------------------ */

void orc_uniform_grid(int ndim, int nb, double *edges) {
  for (int m = 0; m < ndim; ++m)
    for (int b = 0; b <= nb; ++b) edges[(size_t)m * (nb + 1) + b] = (double)b / nb;
}

int orc_fermi_momenta(const orc_problem *pb, double out[3]) {
  orc_medium md;
  medium_of(pb, &md);
  out[0] = md.kF[0];
  out[1] = md.kF[1];
  out[2] = md.Rpart;
  return 0;
}

/* Evaluate samples [first, first+count) of iteration `iter` with the given
 * grid.  w_out[i] = weight, wcond_out[i] = condition scale (may be NULL). */
int orc_sample_values(const orc_problem *pb, const double *edges, uint32_t iter,
                      uint64_t first, uint64_t count, double *w_out,
                      double *wcond_out) {
  if (pb->q == 2 && pb->proton_fraction != 0.0) return -2;
  orc_medium md;
  medium_of(pb, &md);
  if (pb->group >= 0) {
    group_ctx g;
    if (group_setup(pb, &md, &g)) return -1;
    const int nd = 3 * (pb->order + 1);
#pragma omp parallel for schedule(static)
    for (long long i = 0; i < (long long)count; ++i) {
      double x[ORC_MAXDIM], wc;
      int bins[ORC_MAXDIM];
      double jv = vegas_map(nd, pb->n_bins, edges, pb->seed, pb->task_key, iter,
                            first + (uint64_t)i, x, bins);
      double w = group_eval(&g, x, &wc, NULL);
      w_out[i] = jv * w;
      if (wcond_out) wcond_out[i] = fabs(jv) * wc;
    }
    group_free(&g);
    return 0;
  }
  orc_diagram d;
  if (orc_get_diagram(pb->order, pb->diagram_id, &d)) return -1;
  phys_ctx ctx = {pb, &d, &md};
#pragma omp parallel for schedule(static)
  for (long long i = 0; i < (long long)count; ++i) {
    double x[ORC_MAXDIM], wc;
    int bins[ORC_MAXDIM];
    double jv = vegas_map(d.ndim, pb->n_bins, edges, pb->seed, pb->task_key, iter,
                          first + (uint64_t)i, x, bins);
    double w = phys_eval(&ctx, x, &wc, NULL);
    w_out[i] = jv * w;
    if (wcond_out) wcond_out[i] = fabs(jv) * wc;
  }
  return 0;
}

/* Regularised components of samples [first, first+count):
 * wreg_out[i * reg_k + k] (component k + 1, VEGAS Jacobian included). */
int orc_sample_values_reg(const orc_problem *pb, const double *edges, uint32_t iter,
                          uint64_t first, uint64_t count, double *wreg_out) {
  if (pb->reg_k < 1 || pb->reg_k > ORC_MAXREG) return -3;
  if (pb->q == 2 && pb->proton_fraction != 0.0) return -2;
  orc_medium md;
  medium_of(pb, &md);
  const int nd = 3 * (pb->order + 1), K = pb->reg_k;
  group_ctx g;
  orc_diagram d;
  phys_ctx ctx = {pb, &d, &md};
  if (pb->group >= 0) {
    if (group_setup(pb, &md, &g)) return -1;
  } else if (orc_get_diagram(pb->order, pb->diagram_id, &d)) {
    return -1;
  }
#pragma omp parallel for schedule(static)
  for (long long i = 0; i < (long long)count; ++i) {
    double x[ORC_MAXDIM], wr[ORC_MAXREG];
    int bins[ORC_MAXDIM];
    double jv = vegas_map(nd, pb->n_bins, edges, pb->seed, pb->task_key, iter,
                          first + (uint64_t)i, x, bins);
    if (pb->group >= 0) group_eval(&g, x, NULL, wr);
    else phys_eval(&ctx, x, NULL, wr);
    for (int k = 0; k < K; ++k) wreg_out[i * K + k] = jv * wr[k];
  }
  if (pb->group >= 0) group_free(&g);
  return 0;
}

/* VEGAS map alone: x and Jacobian for samples [first, first+count). */
int orc_map_samples(int nd, int nb, const double *edges, uint32_t seed,
                    uint32_t task_key, uint32_t iter, uint64_t first,
                    uint64_t count, double *x_out, double *jac_out,
                    int *bins_out) {
  for (uint64_t i = 0; i < count; ++i) {
    int bins[ORC_MAXDIM];
    jac_out[i] = vegas_map(nd, nb, edges, seed, task_key, iter, first + i,
                           x_out + i * nd, bins);
    if (bins_out)
      for (int m = 0; m < nd; ++m) bins_out[i * nd + m] = bins[m];
  }
  return 0;
}

/* Integrand (single diagram or group, sphere Jacobian included, no VEGAS
 * Jacobian) at explicit hypercube points x[count][3(order+1)]. */
int orc_eval_x(const orc_problem *pb, const double *x, uint64_t count, double *w_out) {
  orc_medium md;
  medium_of(pb, &md);
  const int nd = 3 * (pb->order + 1);
  if (pb->group >= 0) {
    group_ctx g;
    if (group_setup(pb, &md, &g)) return -1;
    for (uint64_t i = 0; i < count; ++i) w_out[i] = group_eval(&g, x + i * nd, NULL, NULL);
    group_free(&g);
    return 0;
  }
  orc_diagram d;
  if (orc_get_diagram(pb->order, pb->diagram_id, &d)) return -1;
  phys_ctx ctx = {pb, &d, &md};
  for (uint64_t i = 0; i < count; ++i) w_out[i] = phys_eval(&ctx, x + i * nd, NULL, NULL);
  return 0;
}

/* Integrand at explicit loop momenta (no Jacobian), for invariance tests. */
int orc_eval_momenta(const orc_problem *pb, const double *kl_flat, double *f_out,
                     double *wcond_out) {
  orc_diagram d;
  if (orc_get_diagram(pb->order, pb->diagram_id, &d)) return -1;
  orc_medium md;
  medium_of(pb, &md);
  orc_point pt;
  eval_point(pb, &d, &md, (const double(*)[3])kl_flat, &pt);
  *f_out = pt.f;
  if (wcond_out) *wcond_out = pt.wcond;
  return 0;
}

/* ------------------------------------------------------------------------ */
/* VEGAS refinement and combination                                          */
/* ------------------------------------------------------------------------ */

/* Lepage refinement of one dimension: hist[b] = sum of w^2 in bin b.
 * Smooth with (7,1)/8, (1,6,1)/8, (1,7)/8, normalize, weight by
 * ((d - 1)/ln d)^alpha, then place new edges so that each new bin holds an
 * equal share of the total weight, the weight being uniform within old bins. */
void orc_refine_dim(int nb, double alpha, const double *hist, double *edges) {
  double ds[ORC_MAXBINS], r[ORC_MAXBINS], xnew[ORC_MAXBINS + 1];
  if (nb < 2) return;
  ds[0] = (7.0 * hist[0] + hist[1]) / 8.0;
  for (int b = 1; b < nb - 1; ++b) ds[b] = (hist[b - 1] + 6.0 * hist[b] + hist[b + 1]) / 8.0;
  ds[nb - 1] = (hist[nb - 2] + 7.0 * hist[nb - 1]) / 8.0;
  double sum = 0.0;
  for (int b = 0; b < nb; ++b) sum += ds[b];
  if (!(sum > 0.0)) return;
  double rtot = 0.0;
  for (int b = 0; b < nb; ++b) {
    double v = ds[b] / sum;
    if (v <= 0.0) r[b] = 0.0;
    else if (v >= 1.0) r[b] = 1.0;
    else r[b] = pow((v - 1.0) / log(v), alpha);
    rtot += r[b];
  }
  if (!(rtot > 0.0)) return;
  double per = rtot / nb;
  xnew[0] = 0.0;
  xnew[nb] = 1.0;
  double acc = 0.0;
  int j = 0;
  for (int k = 1; k < nb; ++k) {
    double target = per * k;
    while (j < nb - 1 && acc + r[j] < target) {
      acc += r[j];
      ++j;
    }
    double frac = r[j] > 0.0 ? (target - acc) / r[j] : 0.0;
    if (frac > 1.0) frac = 1.0;
    if (frac < 0.0) frac = 0.0;
    xnew[k] = edges[j] + frac * (edges[j + 1] - edges[j]);
  }
  for (int b = 0; b <= nb; ++b) edges[b] = xnew[b];
}

typedef struct {
  double mean;      /* inverse-variance weighted mean over iterations */
  double sigma;
  double chi2_dof;
  double last_mean, last_sigma;
  int iters;
  uint64_t n_evals;
} orc_result;

/* Neumaier compensated summation */
typedef struct { double s, c; } ksum;
static void ksum_add(ksum *a, double x) {
  double t = a->s + x;
  if (fabs(a->s) >= fabs(x)) a->c += (a->s - t) + x;
  else a->c += (x - t) + a->s;
  a->s = t;
}
static double ksum_val(const ksum *a) { return a->s + a->c; }

/* Combine iterations: mean = sum(I_k/v_k)/sum(1/v_k), sigma = sum(1/v_k)^-1/2,
 * chi2/dof = sum (I_k - mean)^2/v_k / (K - 1).  Iterations with zero variance
 * are exact: if any, the mean is their plain average and sigma = 0. */
void orc_combine(int K, const double *I, const double *var, orc_result *res) {
  int nzero = 0;
  double zsum = 0.0;
  for (int k = 0; k < K; ++k)
    if (var[k] <= 0.0) { nzero++; zsum += I[k]; }
  res->iters = K;
  if (K == 0) { res->mean = res->sigma = res->chi2_dof = 0.0; return; }
  res->last_mean = I[K - 1];
  res->last_sigma = sqrt(var[K - 1] > 0 ? var[K - 1] : 0.0);
  if (nzero) {
    res->mean = zsum / nzero;
    res->sigma = 0.0;
    res->chi2_dof = 0.0;
    return;
  }
  double wsum = 0, wisum = 0;
  for (int k = 0; k < K; ++k) {
    wsum += 1.0 / var[k];
    wisum += I[k] / var[k];
  }
  res->mean = wisum / wsum;
  res->sigma = sqrt(1.0 / wsum);
  double chi2 = 0.0;
  for (int k = 0; k < K; ++k) chi2 += (I[k] - res->mean) * (I[k] - res->mean) / var[k];
  res->chi2_dof = K > 1 ? chi2 / (K - 1) : 0.0;
}

#define ORC_CHUNK 4096

/* VEGAS iterations over an integrand in the unit hypercube.  Chunks of
 * ORC_CHUNK consecutive samples are summed separately and reduced in chunk
 * order, so results do not depend on the thread count.  The variance sums use
 * the previous iteration's estimate as shift: S1 = sum(w - c),
 * S2 = sum (w - c)^2, I = c + S1/N, var = (S2/N - (S1/N)^2)/(N - 1). */
/* Weights a_k (k = 1..K) of the extrapolation to zero shift: the value at
 * eta = 0 of the least-squares polynomial of degree min(2, K - 1) through the
 * K points (k eta, y_k) with equal weights is sum_k a_k y_k (independent of
 * eta).  Written out as a = first row of (V^T V)^{-1} V^T, V[k][j] = k^j,
 * with the normal equations solved by Gauss-Jordan elimination. */
int orc_extrapolation_weights(int K, double *a) {
  if (K < 1 || K > ORC_MAXREG) return -3;
  const int m = K - 1 < 2 ? K - 1 + 1 : 3;  /* polynomial coefficients */
  double A[3][3] = {{0}}, Inv[3][3] = {{0}};
  for (int i = 0; i < m; ++i)
    for (int j = 0; j < m; ++j)
      for (int k = 1; k <= K; ++k) A[i][j] += pow((double)k, i) * pow((double)k, j);
  for (int i = 0; i < m; ++i) Inv[i][i] = 1.0;
  for (int c = 0; c < m; ++c) {
    int piv = c;
    for (int r = c + 1; r < m; ++r)
      if (fabs(A[r][c]) > fabs(A[piv][c])) piv = r;
    for (int j = 0; j < m; ++j) {
      double t = A[c][j]; A[c][j] = A[piv][j]; A[piv][j] = t;
      t = Inv[c][j]; Inv[c][j] = Inv[piv][j]; Inv[piv][j] = t;
    }
    const double d = A[c][c];
    for (int j = 0; j < m; ++j) { A[c][j] /= d; Inv[c][j] /= d; }
    for (int r = 0; r < m; ++r) {
      if (r == c) continue;
      const double f = A[r][c];
      for (int j = 0; j < m; ++j) { A[r][j] -= f * A[c][j]; Inv[r][j] -= f * Inv[c][j]; }
    }
  }
  for (int k = 1; k <= K; ++k) {
    double v = 0.0;
    for (int j = 0; j < m; ++j) v += Inv[0][j] * pow((double)k, j);
    a[k - 1] = v;
  }
  return 0;
}

/* nreg > 0: the integrand's regularised components are estimated from the
 * same samples (shifted sums with the main component's shift; the grid
 * adapts to the main component), per iteration into Ireg/Vreg[it * (nreg + 1)
 * + k] for component k + 1, and in column nreg the extrapolation to zero
 * shift integrated as an integrand of its own: sum_k a_k w_k per sample
 * (orc_extrapolation_weights), so that its variance carries the components'
 * correlation (they share samples). */
static int vegas_run(int nd, int nb, double alpha, uint32_t seed, uint32_t task_key,
                     integrand_fn fn, const void *ctx, double *edges, uint64_t N,
                     int iters, uint32_t first_iter, int nthreads, double *I_out,
                     double *var_out, orc_result *res, int nreg, double *Ireg,
                     double *Vreg, int train_iters) {
  if (N < 2 || iters < 1 || nd < 1 || nd > ORC_MAXDIM || nb < 2 || nb > ORC_MAXBINS)
    return -3;
  uint64_t nchunks = (N + ORC_CHUNK - 1) / ORC_CHUNK;
  double *chist = calloc((size_t)nchunks * nd * nb, sizeof(double));
  ksum *cs1 = calloc(nchunks, sizeof(ksum));
  ksum *cs2 = calloc(nchunks, sizeof(ksum));
  const int ncol = nreg > 0 ? nreg + 1 : 1;  /* components, then the extrapolation */
  double ax[ORC_MAXREG] = {0};
  if (nreg > 0 && orc_extrapolation_weights(nreg, ax)) return -3;
  ksum *cr1 = calloc(nchunks * ncol, sizeof(ksum));
  ksum *cr2 = calloc(nchunks * ncol, sizeof(ksum));
  double *I = calloc(iters, sizeof(double)), *V = calloc(iters, sizeof(double));
  if (!chist || !cs1 || !cs2 || !cr1 || !cr2 || !I || !V) return -4;
  double shift = 0.0;
#ifdef _OPENMP
  if (nthreads > 0) omp_set_num_threads(nthreads);
#endif
  for (int it = 0; it < iters; ++it) {
    uint32_t iter = first_iter + (uint32_t)it;
    memset(chist, 0, sizeof(double) * (size_t)nchunks * nd * nb);
#pragma omp parallel for schedule(dynamic, 1)
    for (long long c = 0; c < (long long)nchunks; ++c) {
      ksum s1 = {0, 0}, s2 = {0, 0}, r1[ORC_MAXREG + 1], r2[ORC_MAXREG + 1];
      for (int k = 0; k <= ORC_MAXREG; ++k) r1[k] = r2[k] = (ksum){0, 0};
      double *h = chist + (size_t)c * nd * nb;
      uint64_t s0 = (uint64_t)c * ORC_CHUNK;
      uint64_t s1e = s0 + ORC_CHUNK < N ? s0 + ORC_CHUNK : N;
      for (uint64_t s = s0; s < s1e; ++s) {
        double x[ORC_MAXDIM];
        int bins[ORC_MAXDIM];
        double jv = vegas_map(nd, nb, edges, seed, task_key, iter, s, x, bins);
        double wr[ORC_MAXREG];
        double w = jv * fn(ctx, x, NULL, nreg > 0 ? wr : NULL);
        ksum_add(&s1, w - shift);
        ksum_add(&s2, (w - shift) * (w - shift));
        if (nreg > 0) {
          double ex = 0.0;
          for (int k = 0; k < nreg; ++k) {
            const double u = jv * wr[k] - shift;
            ksum_add(&r1[k], u);
            ksum_add(&r2[k], u * u);
            ex += ax[k] * jv * wr[k];
          }
          const double u = ex - shift;
          ksum_add(&r1[nreg], u);
          ksum_add(&r2[nreg], u * u);
        }
        for (int m = 0; m < nd; ++m) h[m * nb + bins[m]] += w * w;
      }
      cs1[c] = s1;
      cs2[c] = s2;
      for (int k = 0; k < ncol && nreg > 0; ++k) {
        cr1[c * ncol + k] = r1[k];
        cr2[c * ncol + k] = r2[k];
      }
    }
    for (int k = 0; k < ncol && nreg > 0; ++k) {
      ksum R1 = {0, 0}, R2 = {0, 0};
      for (uint64_t c = 0; c < nchunks; ++c) {
        ksum_add(&R1, ksum_val(&cr1[c * ncol + k]));
        ksum_add(&R2, ksum_val(&cr2[c * ncol + k]));
      }
      const double q1 = ksum_val(&R1) / (double)N, q2 = ksum_val(&R2) / (double)N;
      double v = (q2 - q1 * q1) / (double)(N - 1);
      if (v < 0.0) v = 0.0;
      if (Ireg) Ireg[(size_t)it * ncol + k] = shift + q1;
      if (Vreg) Vreg[(size_t)it * ncol + k] = v;
    }
    ksum S1 = {0, 0}, S2 = {0, 0};
    for (uint64_t c = 0; c < nchunks; ++c) {
      ksum_add(&S1, ksum_val(&cs1[c]));
      ksum_add(&S2, ksum_val(&cs2[c]));
    }
    double m1 = ksum_val(&S1) / (double)N;
    double m2 = ksum_val(&S2) / (double)N;
    double var = (m2 - m1 * m1) / (double)(N - 1);
    if (var < 0.0) var = 0.0;
    I[it] = shift + m1;
    V[it] = var;
    /* training phase: adapt; evaluation phase: the grid stays frozen */
    const int adapt = train_iters <= 0 || it < train_iters;
    for (int m = 0; m < nd && adapt; ++m) {
      double hist[ORC_MAXBINS];
      for (int b = 0; b < nb; ++b) {
        double s = 0.0;
        for (uint64_t c = 0; c < nchunks; ++c) s += chist[(size_t)c * nd * nb + m * nb + b];
        hist[b] = s;
      }
      orc_refine_dim(nb, alpha, hist, edges + (size_t)m * (nb + 1));
    }
    shift = I[it];
  }
  /* with a training phase, the evaluation iterations alone (once there are
   * any) make the combined estimate */
  if (train_iters > 0 && iters > train_iters)
    orc_combine(iters - train_iters, I + train_iters, V + train_iters, res);
  else
    orc_combine(iters, I, V, res);
  res->n_evals = N * (uint64_t)iters;
  if (I_out) memcpy(I_out, I, sizeof(double) * iters);
  if (var_out) memcpy(var_out, V, sizeof(double) * iters);
  free(chist); free(cs1); free(cs2); free(cr1); free(cr2); free(I); free(V);
  return 0;
}

/* Full VEGAS run of one diagram at one EOS point. */
int orc_integrate_reg(const orc_problem *pb, double *edges, uint64_t N, int iters,
                      uint32_t first_iter, int nthreads, double *I_out, double *var_out,
                      orc_result *res, double *Ireg, double *Vreg) {
  const int nreg = pb->reg_k > ORC_MAXREG ? ORC_MAXREG : pb->reg_k;
  if (pb->q == 2 && pb->proton_fraction != 0.0) return -2;
  orc_medium md;
  medium_of(pb, &md);
  if (pb->group >= 0) {
    group_ctx g;
    if (group_setup(pb, &md, &g)) return -1;
    int rc = vegas_run(3 * (pb->order + 1), pb->n_bins, pb->alpha, pb->seed, pb->task_key,
                       group_eval, &g, edges, N, iters, first_iter, nthreads, I_out, var_out,
                       res, nreg, Ireg, Vreg, pb->train_iters);
    group_free(&g);
    return rc;
  }
  orc_diagram d;
  if (orc_get_diagram(pb->order, pb->diagram_id, &d)) return -1;
  phys_ctx ctx = {pb, &d, &md};
  return vegas_run(d.ndim, pb->n_bins, pb->alpha, pb->seed, pb->task_key, phys_eval,
                   &ctx, edges, N, iters, first_iter, nthreads, I_out, var_out, res, nreg, Ireg,
                   Vreg, pb->train_iters);
}

/* Full VEGAS run of one diagram (or group) at one EOS point. */
int orc_integrate(const orc_problem *pb, double *edges, uint64_t N, int iters,
                  uint32_t first_iter, int nthreads, double *I_out,
                  double *var_out, orc_result *res) {
  orc_problem p = *pb;
  p.reg_k = 0;
  return orc_integrate_reg(&p, edges, N, iters, first_iter, nthreads, I_out, var_out, res, NULL,
                           NULL);
}


/* VEGAS run of the separable Gaussian test integrand. */
int orc_integrate_gaussian(int nd, double width, int nb, double alpha, uint32_t seed,
                           uint32_t task_key, double *edges, uint64_t N, int iters,
                           int nthreads, double *I_out, double *var_out,
                           orc_result *res) {
  gauss_ctx g = {width, nd};
  return vegas_run(nd, nb, alpha, seed, task_key, gauss_eval, &g, edges, N, iters, 0,
                   nthreads, I_out, var_out, res, 0, NULL, NULL, 0);
}

int orc_max_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}
