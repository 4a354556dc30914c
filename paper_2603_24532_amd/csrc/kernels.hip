// HIP kernels for gfx950 (CDNA4): VEGAS Monte Carlo of MBPT energy diagrams.
//
// One thread evaluates one sample at a time: Philox4x32-10 words -> VEGAS
// bins and fractions (grid in LDS) -> spherical loop momenta -> line momenta
// from the compiled descriptor -> Pauli factors (n_k for holes, 1 - n_k for
// particles) -> energy denominators (Eq. (6), free spectrum) ->
// antisymmetrised matrix elements per vertex -> explicit spin(-isospin) label
// sum -> weight.  Sums of (w - c) and (w - c)^2 are kept per thread with
// Neumaier compensation, reduced across the wavefront and the block in a
// fixed order and written per work item; refinement histograms of w^2 are
// privatised in LDS and merged with fp64 atomics.  The integrand is
// elementwise with no contraction, so it runs on the vector ALUs (no MFMA).
#include <hip/hip_runtime.h>

#include "device_types.hpp"
#include "kernels.hpp"

namespace mbpt {

// ---------------------------------------------------------------------------
// Philox4x32-10 (Salmon et al., SC'11)

__device__ __forceinline__ void philox4x32_10(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3,
                                              uint32_t k0, uint32_t k1, uint32_t *out) {
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    const uint32_t hi0 = __umulhi(0xD2511F53u, c0), lo0 = 0xD2511F53u * c0;
    const uint32_t hi1 = __umulhi(0xCD9E8D57u, c2), lo1 = 0xCD9E8D57u * c2;
    const uint32_t n0 = hi1 ^ c1 ^ k0;
    const uint32_t n2 = hi0 ^ c3 ^ k1;
    c0 = n0;
    c1 = lo1;
    c2 = n2;
    c3 = lo0;
    k0 += 0x9E3779B9u;
    k1 += 0xBB67AE85u;
  }
  out[0] = c0;
  out[1] = c1;
  out[2] = c2;
  out[3] = c3;
}

// Neumaier step: (s, c) += x
__device__ __forceinline__ void neumaier(double &s, double &c, double x) {
  const double t = s + x;
  c += (fabs(s) >= fabs(x)) ? ((s - t) + x) : ((x - t) + s);
  s = t;
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

template <int ORDER, int Q>
__device__ __forceinline__ double eval_fp64(const KArgs &a, const TaskDev *__restrict__ T,
                                            const DiagDev *__restrict__ D,
                                            const double2 *__restrict__ g, uint64_t s,
                                            uint32_t iter, int *bins, uint32_t &npass,
                                            uint32_t &nterms) {
  constexpr int L = ORDER + 1;
  constexpr int NL = 2 * ORDER;
  constexpr int NC = ORDER - 1;
  constexpr int ND = 3 * L;
  constexpr int NW = (ND + 3) / 4;
  const int nb = a.phys.nb;

  // Philox words: counter (s lo, s hi, iteration, word block), key (seed, task)
  uint32_t wd[4 * NW];
#pragma unroll
  for (int j = 0; j < NW; ++j)
    philox4x32_10(static_cast<uint32_t>(s), static_cast<uint32_t>(s >> 32), iter,
                  static_cast<uint32_t>(j), a.phys.seed, T->key, wd + 4 * j);

  // VEGAS map: bin b = floor(w nb / 2^32), fraction ((w nb mod 2^32) + 1/2) / 2^32
  double x[ND];
  double jac = 1.0;
#pragma unroll
  for (int m = 0; m < ND; ++m) {
    const uint32_t w = wd[m];
    const int b = static_cast<int>(__umulhi(w, static_cast<uint32_t>(nb)));
    const uint32_t lo = w * static_cast<uint32_t>(nb);
    const double r = (static_cast<double>(lo) + 0.5) * 0x1p-32;
    const double2 ew = g[m * nb + b];
    x[m] = ew.x + r * ew.y;
    jac *= static_cast<double>(nb) * ew.y;
    bins[m] = b;
  }

  // loop momenta: radius R x0, cos theta = 2 x1 - 1, azimuth 2 pi x2
  double k[L][3];
#pragma unroll
  for (int j = 0; j < L; ++j) {
    const double R = D->loop_part[j] ? T->Rp : T->Rh;
    const double rad = R * x[3 * j];
    const double ct = 2.0 * x[3 * j + 1] - 1.0;
    const double st = sqrt(fmax(0.0, (1.0 - ct) * (1.0 + ct)));
    double sp, cp;
    sincospi(2.0 * x[3 * j + 2], &sp, &cp);
    k[j][0] = rad * st * cp;
    k[j][1] = rad * st * sp;
    k[j][2] = rad * ct;
    jac *= R * rad * rad * (4.0 * M_PI);
  }

  // line momenta -> occupation tests and energies
  double eps[NL];
  uint32_t inN = 0, inP = 0;
#pragma unroll
  for (int l = 0; l < NL; ++l) {
    double kx = 0.0, ky = 0.0, kz = 0.0;
#pragma unroll
    for (int j = 0; j < L; ++j) {
      const double c = D->lc[l][j];
      kx = fma(c, k[j][0], kx);
      ky = fma(c, k[j][1], ky);
      kz = fma(c, k[j][2], kz);
    }
    const double k2 = kx * kx + ky * ky + kz * kz;
    eps[l] = a.phys.hb2m * k2;
    inN |= (k2 < T->kF2[0]) ? (1u << l) : 0u;
    if (Q == 4) inP |= (k2 < T->kF2[1]) ? (1u << l) : 0u;
  }
  // a hole line is allowed if occupied, a particle line if empty
  const uint32_t lmask = D->line_mask, pmask = D->part_mask;
  const uint32_t okN = (inN ^ pmask) & lmask;
  const uint32_t okP = (inP ^ pmask) & lmask;
  if (Q == 2 && okN != lmask) return 0.0;
  ++npass;

  // energy denominators
  double dprod = 1.0;
#pragma unroll
  for (int c = 0; c < NC; ++c) {
    double Dc = 0.0;
#pragma unroll
    for (int l = 0; l < NL; ++l) Dc = fma(D->cutc[c][l], eps[l], Dc);
    dprod *= Dc;
  }

  // antisymmetrised matrix elements: V_d = V(p, p'), V_e = V(p, -p')
  double Vd[ORDER], Ve[ORDER];
#pragma unroll
  for (int v = 0; v < ORDER; ++v) {
    double p[3] = {0.0, 0.0, 0.0}, q[3] = {0.0, 0.0, 0.0};
#pragma unroll
    for (int j = 0; j < L; ++j) {
      const double cp = D->vp[v][j], cq = D->vq[v][j];
#pragma unroll
      for (int i = 0; i < 3; ++i) {
        p[i] = fma(cp, k[j][i], p[i]);
        q[i] = fma(cq, k[j][i], q[i]);
      }
    }
    const double p2 = p[0] * p[0] + p[1] * p[1] + p[2] * p[2];
    const double q2 = q[0] * q[0] + q[1] * q[1] + q[2] * q[2];
    const double pq = p[0] * q[0] + p[1] * q[1] + p[2] * q[2];
    double pn = p2, qn = q2;
    for (int e = 1; e < a.phys.half_exp; ++e) {
      pn *= p2;
      qn *= q2;
    }
    const double reg = exp(-(pn + qn) * a.phys.invLn);
    const double s2 = p2 + q2 + a.phys.m2;
    Vd[v] = reg * (a.phys.V0 + a.phys.Vy / (s2 - 2.0 * pq));
    Ve[v] = reg * (a.phys.V0 + a.phys.Vy / (s2 + 2.0 * pq));
  }

  // label sum: isospin groups (Pauli test per group), terms with multiplicity
  double acc = 0.0;
  const GroupDev *__restrict__ G = a.groups + D->group_off;
  const int ngroups = D->ngroups;
  for (int gi = 0; gi < ngroups; ++gi) {
    const uint32_t tau = G[gi].tau;
    const int first = G[gi].first, cnt = G[gi].count;
    bool ok = true;
    if (Q == 4) ok = (((~tau & ~okN) | (tau & ~okP)) & lmask) == 0u;
    if (ok) {
      nterms += cnt;
      for (int t = first; t < first + cnt; ++t) {
        const TermDev tm = a.terms[t];
        double prod = 1.0;
#pragma unroll
        for (int v = 0; v < ORDER; ++v) {
          const uint32_t code = (tm.codes >> (2 * v)) & 3u;
          const double ca = code != 1u ? 1.0 : 0.0;
          const double cb = code != 0u ? -1.0 : 0.0;
          prod *= fma(ca, Vd[v], cb * Ve[v]);
        }
        acc = fma(tm.mult, prod, acc);
      }
    }
  }
  return jac * (D->pref * T->inv_density) * acc / dprod;
}

// ---------------------------------------------------------------------------
// Work item: blockDim.x * spt consecutive samples of one task

template <int ORDER, int Q>
__device__ __forceinline__ void process_item(const KArgs &a, int t, int item, double *smem) {
  constexpr int ND = 3 * (ORDER + 1);
  const TaskDev *__restrict__ T = a.tasks + t;
  const DiagDev *__restrict__ D = a.diags + T->diag;
  const int nb = a.phys.nb;
  const int tid = threadIdx.x, bs = blockDim.x;
  double2 *g = reinterpret_cast<double2 *>(smem);
  double *h = smem + 2 * ND * nb;
  double *red = h + ND * nb;

  __syncthreads();  // previous item done with LDS
  const double *ge = a.grids + T->grid_off;
  for (int i = tid; i < ND * nb; i += bs) {
    const int m = i / nb, b = i - m * nb;
    const double e0 = ge[m * (nb + 1) + b], e1 = ge[m * (nb + 1) + b + 1];
    g[i] = make_double2(e0, e1 - e0);
    h[i] = 0.0;
  }
  __syncthreads();

  const uint64_t N = T->nsamples;
  const uint32_t iter = T->iter;
  const double shift = T->shift;
  const uint64_t base = static_cast<uint64_t>(item - T->item_begin) * bs * a.spt;
  double s1 = 0.0, c1 = 0.0, s2 = 0.0, c2 = 0.0;
  uint32_t npass = 0, nterms = 0;
  for (int kk = 0; kk < a.spt; ++kk) {
    const uint64_t s = base + static_cast<uint64_t>(kk) * bs + tid;
    if (s < N) {
      int bins[ND];
      const double w = eval_fp64<ORDER, Q>(a, T, D, g, s, iter, bins, npass, nterms);
      const double d = w - shift;
      neumaier(s1, c1, d);
      neumaier(s2, c2, d * d);
      const double w2 = w * w;
      if (w2 != 0.0) {
#pragma unroll
        for (int m = 0; m < ND; ++m) atomicAdd(&h[m * nb + bins[m]], w2);
      }
    }
  }
  // wavefront butterfly, then waves in order
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) {
    const double os1 = __shfl_xor(s1, off, 64), oc1 = __shfl_xor(c1, off, 64);
    const double os2 = __shfl_xor(s2, off, 64), oc2 = __shfl_xor(c2, off, 64);
    pair_merge(s1, c1, os1, oc1);
    pair_merge(s2, c2, os2, oc2);
    npass += __shfl_xor(npass, off, 64);
    nterms += __shfl_xor(nterms, off, 64);
  }
  const int wave = tid >> 6, lane = tid & 63;
  uint32_t *ured = reinterpret_cast<uint32_t *>(red + 4 * (bs >> 6));
  if (lane == 0) {
    red[4 * wave + 0] = s1;
    red[4 * wave + 1] = c1;
    red[4 * wave + 2] = s2;
    red[4 * wave + 3] = c2;
    ured[2 * wave] = npass;
    ured[2 * wave + 1] = nterms;
  }
  __syncthreads();
  if (tid == 0) {
    double S1 = red[0], C1 = red[1], S2 = red[2], C2 = red[3];
    uint64_t P1 = ured[0], P2 = ured[1];
    for (int w = 1; w < (bs >> 6); ++w) {
      pair_merge(S1, C1, red[4 * w + 0], red[4 * w + 1]);
      pair_merge(S2, C2, red[4 * w + 2], red[4 * w + 3]);
      P1 += ured[2 * w];
      P2 += ured[2 * w + 1];
    }
    double *P = a.partials + 4 * static_cast<size_t>(item);
    P[0] = S1;
    P[1] = C1;
    P[2] = S2;
    P[3] = C2;
    uint64_t *K = a.counters + kItemCounters * static_cast<size_t>(item);
    K[0] = 0;
    K[1] = P1;
    K[2] = P2;
  }
  __syncthreads();
  double *hg = a.hists + T->hist_off;
  for (int i = tid; i < ND * nb; i += bs) {
    const double v = h[i];
    if (v != 0.0) atomicAdd(&hg[i], v);
  }
}

// One task per launch: block b processes work item item_begin + b.
template <int ORDER, int Q>
__global__ __launch_bounds__(256) void sample_single(KArgs a, int t) {
  extern __shared__ double smem[];
  process_item<ORDER, Q>(a, t, a.tasks[t].item_begin + blockIdx.x, smem);
}

// Persistent launch over all work items of all tasks (items grouped by task).
template <int Q>
__global__ __launch_bounds__(256) void sample_batched(KArgs a) {
  extern __shared__ double smem[];
  for (int item = blockIdx.x; item < a.total_items; item += gridDim.x) {
    int lo = 0, hi = a.ntasks - 1;  // last task with item_begin <= item
    while (lo < hi) {
      const int mid = (lo + hi + 1) >> 1;
      if (a.tasks[mid].item_begin <= item) lo = mid;
      else hi = mid - 1;
    }
    const int t = lo;
    switch (a.tasks[t].order) {
      case 1: process_item<1, Q>(a, t, item, smem); break;
      case 2: process_item<2, Q>(a, t, item, smem); break;
      case 3: process_item<3, Q>(a, t, item, smem); break;
      case 4: process_item<4, Q>(a, t, item, smem); break;
      default: process_item<5, Q>(a, t, item, smem); break;
    }
  }
}

// ---------------------------------------------------------------------------
// Iteration end: fixed-order reduction of the item partials, estimate and
// variance, running inverse-variance sums, and Lepage refinement of the grid.

__device__ void refine_dim(double *hist, double *edges, int nb, double alpha, double *ds,
                           double *r, double *xnew) {
  ds[0] = (7.0 * hist[0] + hist[1]) / 8.0;
  for (int b = 1; b < nb - 1; ++b) ds[b] = (hist[b - 1] + 6.0 * hist[b] + hist[b + 1]) / 8.0;
  ds[nb - 1] = (hist[nb - 2] + 7.0 * hist[nb - 1]) / 8.0;
  double sum = 0.0;
  for (int b = 0; b < nb; ++b) sum += ds[b];
  if (!(sum > 0.0)) return;
  double rtot = 0.0;
  for (int b = 0; b < nb; ++b) {
    const double v = ds[b] / sum;
    double rb;
    if (v <= 0.0) rb = 0.0;
    else if (v >= 1.0) rb = 1.0;
    else rb = pow((v - 1.0) / log(v), alpha);
    r[b] = rb;
    rtot += rb;
  }
  if (!(rtot > 0.0)) return;
  const double per = rtot / nb;
  xnew[0] = 0.0;
  xnew[nb] = 1.0;
  double acc = 0.0;
  int j = 0;
  for (int kk = 1; kk < nb; ++kk) {
    const double target = per * kk;
    while (j < nb - 1 && acc + r[j] < target) {
      acc += r[j];
      ++j;
    }
    double frac = r[j] > 0.0 ? (target - acc) / r[j] : 0.0;
    frac = fmin(1.0, fmax(0.0, frac));
    xnew[kk] = edges[j] + frac * (edges[j + 1] - edges[j]);
  }
  for (int b = 0; b <= nb; ++b) edges[b] = xnew[b];
}

__global__ __launch_bounds__(256) void finish_iteration(KArgs a, int first_task, double alpha) {
  __shared__ double red[4 * 4];
  __shared__ unsigned long long kred[4][kItemCounters];
  extern __shared__ double scratch[];
  const int t = first_task + blockIdx.x;
  TaskDev *T = a.tasks + t;
  if (!T->active) return;
  const int tid = threadIdx.x, bs = blockDim.x;
  double s1 = 0.0, c1 = 0.0, s2 = 0.0, c2 = 0.0;
  unsigned long long kc[kItemCounters] = {0, 0, 0};
  for (int it = T->item_begin + tid; it < T->item_begin + T->nitems; it += bs) {
    const double *P = a.partials + 4 * static_cast<size_t>(it);
    pair_merge(s1, c1, P[0], P[1]);
    pair_merge(s2, c2, P[2], P[3]);
    for (int j = 0; j < kItemCounters; ++j) kc[j] += a.counters[kItemCounters * static_cast<size_t>(it) + j];
  }
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) {
    const double os1 = __shfl_xor(s1, off, 64), oc1 = __shfl_xor(c1, off, 64);
    const double os2 = __shfl_xor(s2, off, 64), oc2 = __shfl_xor(c2, off, 64);
    pair_merge(s1, c1, os1, oc1);
    pair_merge(s2, c2, os2, oc2);
    for (int j = 0; j < kItemCounters; ++j) kc[j] += __shfl_xor(kc[j], off, 64);
  }
  const int wave = tid >> 6, lane = tid & 63;
  if (lane == 0) {
    red[4 * wave + 0] = s1;
    red[4 * wave + 1] = c1;
    red[4 * wave + 2] = s2;
    red[4 * wave + 3] = c2;
    for (int j = 0; j < kItemCounters; ++j) kred[wave][j] = kc[j];
  }
  __syncthreads();
  if (tid == 0) {
    double S1 = red[0], C1 = red[1], S2 = red[2], C2 = red[3];
    unsigned long long F[kItemCounters] = {kred[0][0], kred[0][1], kred[0][2]};
    for (int w = 1; w < (bs >> 6); ++w) {
      pair_merge(S1, C1, red[4 * w + 0], red[4 * w + 1]);
      pair_merge(S2, C2, red[4 * w + 2], red[4 * w + 3]);
      for (int j = 0; j < kItemCounters; ++j) F[j] += kred[w][j];
    }
    const double N = static_cast<double>(T->nsamples);
    const double m1 = (S1 + C1) / N;
    const double m2 = (S2 + C2) / N;
    double var = (m2 - m1 * m1) / (N - 1.0);
    if (var < 0.0) var = 0.0;
    const double I = T->shift + m1;
    if (T->res_cap > 0) {
      double *lg = a.reslog + 2 * (T->res_off + (T->it_done % T->res_cap));
      lg[0] = I;
      lg[1] = var;
    }
    if (var > 0.0) {
      T->wsum += 1.0 / var;
      T->wisum += I / var;
      T->wi2sum += I * I / var;
    } else {
      T->nzero += 1;
      T->zsum += I;
    }
    T->lastI = I;
    T->lastV = var;
    T->shift = I;
    T->iter += 1;
    T->it_done += 1;
    T->nevals += T->nsamples;
    T->nfallback += F[0];
    T->npass += F[1];
    T->nterms += F[2];
  }
  // refinement: one thread per dimension, scratch in LDS
  const int nb = a.phys.nb;
  for (int m = tid; m < T->nd; m += bs) {
    double *ds = scratch + static_cast<size_t>(m) * (3 * nb + 1);
    double *hist = a.hists + T->hist_off + m * nb;
    double *edges = a.grids + T->grid_off + m * (nb + 1);
    refine_dim(hist, edges, nb, alpha, ds, ds + nb, ds + 2 * nb);
    for (int b = 0; b < nb; ++b) hist[b] = 0.0;
  }
}

// ---------------------------------------------------------------------------
// Per-sample dump for parity checks: thread i evaluates sample first + i.

template <int ORDER, int Q>
__global__ __launch_bounds__(256) void dump_samples(KArgs a, int t, uint32_t iter, uint64_t first,
                                                   uint64_t count, double *out) {
  extern __shared__ double smem[];
  constexpr int ND = 3 * (ORDER + 1);
  const TaskDev *T = a.tasks + t;
  const DiagDev *D = a.diags + T->diag;
  const int nb = a.phys.nb;
  double2 *g = reinterpret_cast<double2 *>(smem);
  const double *ge = a.grids + T->grid_off;
  for (int i = threadIdx.x; i < ND * nb; i += blockDim.x) {
    const int m = i / nb, b = i - m * nb;
    const double e0 = ge[m * (nb + 1) + b], e1 = ge[m * (nb + 1) + b + 1];
    g[i] = make_double2(e0, e1 - e0);
  }
  __syncthreads();
  const uint64_t i = static_cast<uint64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < count) {
    int bins[ND];
    uint32_t np = 0, nt = 0;
    out[i] = eval_fp64<ORDER, Q>(a, T, D, g, first + i, iter, bins, np, nt);
  }
}

// Reset grids to uniform, histograms and running state to zero.
__global__ void init_tasks(KArgs a) {
  TaskDev *T = a.tasks + blockIdx.x;
  const int nb = a.phys.nb;
  for (int i = threadIdx.x; i < T->nd * (nb + 1); i += blockDim.x) {
    const int b = i % (nb + 1);
    a.grids[T->grid_off + i] = static_cast<double>(b) / nb;
  }
  for (int i = threadIdx.x; i < T->nd * nb; i += blockDim.x) a.hists[T->hist_off + i] = 0.0;
  if (threadIdx.x == 0) {
    T->iter = 0;
    T->it_done = 0;
    T->shift = 0.0;
    T->wsum = T->wisum = T->wi2sum = T->zsum = 0.0;
    T->nzero = 0;
    T->lastI = T->lastV = 0.0;
    T->nevals = T->nfallback = T->npass = T->nterms = 0;
  }
}

// ---------------------------------------------------------------------------
// Host-side launchers

size_t sample_lds_bytes(int nd, int nb, int block) {
  return (3 * static_cast<size_t>(nd) * nb + 5 * (block / 64)) * sizeof(double);
}

template <int Q>
static hipError_t single_q(const KArgs &a, int t, int order, int nitems, int block,
                           hipStream_t st) {
  const size_t lds = sample_lds_bytes(3 * (order + 1), a.phys.nb, block);
  switch (order) {
    case 1: hipLaunchKernelGGL((sample_single<1, Q>), dim3(nitems), dim3(block), lds, st, a, t); break;
    case 2: hipLaunchKernelGGL((sample_single<2, Q>), dim3(nitems), dim3(block), lds, st, a, t); break;
    case 3: hipLaunchKernelGGL((sample_single<3, Q>), dim3(nitems), dim3(block), lds, st, a, t); break;
    case 4: hipLaunchKernelGGL((sample_single<4, Q>), dim3(nitems), dim3(block), lds, st, a, t); break;
    case 5: hipLaunchKernelGGL((sample_single<5, Q>), dim3(nitems), dim3(block), lds, st, a, t); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_sample_single(const KArgs &a, int t, int order, int q, int nitems, int block,
                                hipStream_t st) {
  return q == 4 ? single_q<4>(a, t, order, nitems, block, st)
                : single_q<2>(a, t, order, nitems, block, st);
}

hipError_t launch_sample_batched(const KArgs &a, int q, int max_nd, int grid, int block,
                                 hipStream_t st) {
  const size_t lds = sample_lds_bytes(max_nd, a.phys.nb, block);
  if (q == 4) hipLaunchKernelGGL((sample_batched<4>), dim3(grid), dim3(block), lds, st, a);
  else hipLaunchKernelGGL((sample_batched<2>), dim3(grid), dim3(block), lds, st, a);
  return hipGetLastError();
}

hipError_t launch_finish(const KArgs &a, int first_task, int ntasks, int max_nd, double alpha,
                         hipStream_t st) {
  const size_t lds = static_cast<size_t>(max_nd) * (3 * a.phys.nb + 1) * sizeof(double);
  hipLaunchKernelGGL(finish_iteration, dim3(ntasks), dim3(256), lds, st, a, first_task, alpha);
  return hipGetLastError();
}

template <int Q>
static hipError_t dump_q(const KArgs &a, int t, int order, uint32_t iter, uint64_t first,
                         uint64_t count, double *out, hipStream_t st) {
  const int block = 256;
  const dim3 grid(static_cast<unsigned>((count + block - 1) / block));
  const size_t lds = 2 * static_cast<size_t>(3 * (order + 1)) * a.phys.nb * sizeof(double);
  switch (order) {
    case 1: hipLaunchKernelGGL((dump_samples<1, Q>), grid, dim3(block), lds, st, a, t, iter, first, count, out); break;
    case 2: hipLaunchKernelGGL((dump_samples<2, Q>), grid, dim3(block), lds, st, a, t, iter, first, count, out); break;
    case 3: hipLaunchKernelGGL((dump_samples<3, Q>), grid, dim3(block), lds, st, a, t, iter, first, count, out); break;
    case 4: hipLaunchKernelGGL((dump_samples<4, Q>), grid, dim3(block), lds, st, a, t, iter, first, count, out); break;
    case 5: hipLaunchKernelGGL((dump_samples<5, Q>), grid, dim3(block), lds, st, a, t, iter, first, count, out); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_dump(const KArgs &a, int t, int order, int q, uint32_t iter, uint64_t first,
                       uint64_t count, double *out, hipStream_t st) {
  return q == 4 ? dump_q<4>(a, t, order, iter, first, count, out, st)
                : dump_q<2>(a, t, order, iter, first, count, out, st);
}

int batched_occupancy(int q, int block, size_t lds) {
  int n = 0;
  const hipError_t e =
      q == 4 ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, sample_batched<4>, block, lds)
             : hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, sample_batched<2>, block, lds);
  return e == hipSuccess ? n : 1;
}

hipError_t launch_init(const KArgs &a, int ntasks, hipStream_t st) {
  hipLaunchKernelGGL(init_tasks, dim3(ntasks), dim3(256), 0, st, a);
  return hipGetLastError();
}

}  // namespace mbpt
