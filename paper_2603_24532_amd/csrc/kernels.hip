// HIP kernels for gfx950 (CDNA4): VEGAS Monte Carlo of MBPT energy diagrams.
//
// One thread evaluates one sample at a time: Philox4x32-10 words -> VEGAS
// bins and fractions (grid in LDS) -> spherical loop momenta -> line momenta
// from the compiled descriptor -> Pauli factors (n_k for holes, 1 - n_k for
// particles) -> energy denominators (eq:Dijkabc, free spectrum) ->
// antisymmetrised matrix elements per vertex -> explicit spin(-isospin) label
// sum -> weight.  Sums of (w - c) and (w - c)^2 are kept per thread as plain
// sums (at most spt terms), merged across the wavefront, the block and the
// work items with compensated pair merges in a fixed order; refinement
// histograms of w^2 are privatised in LDS and merged with fp64 atomics.  The
// integrand is elementwise with no contraction, so it runs on the vector ALUs
// (no MFMA).
//
// This file: the iteration-end, HF-table and init kernels and the launchers;
// the sample kernels are templates in kernels_dev.hpp, instantiated per
// (order, matter) by kernels_inst.hip.
#include "kernels_dev.hpp"

namespace mbpt {

// ---------------------------------------------------------------------------
// Iteration end: fixed-order reduction of the item partials, estimate and
// variance, running inverse-variance sums, and Lepage refinement of the grid.

// Wave-cooperative sum: every lane receives the total (fixed butterfly order).
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// Lepage refinement of one dimension by one wavefront (lanes own bins b and
// b + 64).  hist: sums of w^2 per bin; edges: nb + 1 edges, rewritten.
// Smoothing (7,1)/8, (1,6,1)/8, (1,7)/8, normalisation, compression
// ((d - 1)/ln d)^alpha, then new edges placing an equal share of the total
// compressed weight in every new bin (weight uniform inside old bins).
// scr: 2 nb + 2 doubles of LDS for this wave.
__device__ void refine_dim_wave(double *hist, double *edges, int nb, double alpha, double *scr) {
  const int lane = threadIdx.x & 63;
  double *cum = scr;            // nb + 1 prefix sums of r
  double *r = scr + nb + 1;     // nb compressed weights
  double dsv[2] = {0.0, 0.0};
  double part = 0.0;
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    const int b = lane + 64 * h;
    if (b < nb) {
      double d;
      if (b == 0) d = (7.0 * hist[0] + hist[1]) / 8.0;
      else if (b == nb - 1) d = (hist[nb - 2] + 7.0 * hist[nb - 1]) / 8.0;
      else d = (hist[b - 1] + 6.0 * hist[b] + hist[b + 1]) / 8.0;
      dsv[h] = d;
      part += d;
    }
  }
  const double sum = wave_sum(part);
  if (!(sum > 0.0)) return;  // uniform across the wave
  double rp = 0.0;
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    const int b = lane + 64 * h;
    if (b < nb) {
      const double v = dsv[h] / sum;
      double rb;
      if (v <= 0.0) rb = 0.0;
      else if (v >= 1.0) rb = 1.0;
      else rb = pow((v - 1.0) / log(v), alpha);
      r[b] = rb;
      rp += rb;
    }
  }
  const double rtot = wave_sum(rp);
  if (!(rtot > 0.0)) return;
  __builtin_amdgcn_wave_barrier();
  // inclusive scan over bins 0..63, then 64..127 offset by the first half
  double carry = 0.0;
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    const int b = lane + 64 * h;
    double x = (b < nb) ? r[b] : 0.0;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
      const double y = __shfl_up(x, off, 64);
      if (lane >= off) x += y;
    }
    if (b < nb) cum[b + 1] = carry + x;
    carry += __shfl(x, 63, 64);
  }
  if (lane == 0) cum[0] = 0.0;
  __builtin_amdgcn_wave_barrier();
  __syncwarp();
  const double per = rtot / nb;
  double xnew[2];
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    const int kk = lane + 64 * h;
    xnew[h] = 0.0;
    if (kk >= 1 && kk < nb) {
      const double target = per * kk;
      // smallest j with cum[j + 1] >= target (j = nb - 1 if none)
      int lo = 0, hi = nb - 1;
      while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if (cum[mid + 1] >= target) hi = mid;
        else lo = mid + 1;
      }
      const int j = lo;
      double frac = r[j] > 0.0 ? (target - cum[j]) / r[j] : 0.0;
      frac = fmin(1.0, fmax(0.0, frac));
      xnew[h] = edges[j] + frac * (edges[j + 1] - edges[j]);
    }
  }
  __syncwarp();
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    const int kk = lane + 64 * h;
    if (kk >= 1 && kk < nb) edges[kk] = xnew[h];
  }
}

// step_iter: index of this iteration within the launch sequence; tasks whose
// plan ends before it sit this iteration out.
// One block of kFinishThreads per task: every thread reduces a strided set of
// item partials (loads of kFinishBatch items issued together, merged in item
// order), then the waves reduce in order and each wave refines dimensions.
__global__ __launch_bounds__(kFinishThreads) void finish_iteration(KArgs a, int first_task,
                                                                   double alpha, int step_iter) {
  constexpr int NW = kFinishThreads / 64;
  __shared__ double red[NW * 4];
  __shared__ unsigned long long kred[NW][kItemCounters];
  __shared__ double cred[NW][kRegSums];
  extern __shared__ double scratch[];
  const int t = first_task + blockIdx.x;
  TaskDev *T = a.tasks + t;
  // the persistent launches of the next iteration claim items from zero
  if (a.queue && blockIdx.x == 0 && threadIdx.x < kQueueSlots) a.queue[threadIdx.x] = 0;
  if (!T->active || T->plan <= step_iter) return;
  const int tid = threadIdx.x, bs = blockDim.x;
  const int it0 = T->store_begin, it1 = T->store_begin + T->nitems;
  // regularised components (same samples, main component's shift): item
  // sums in item order per thread, then across the block
  if (a.nreg > 0) {
    double cs[kRegSums];
#pragma unroll
    for (int j = 0; j < kRegSums; ++j) cs[j] = 0.0;
    for (int it = it0 + tid; it < it1; it += bs) {
      const double *C = a.cpart + kRegSums * static_cast<size_t>(it);
#pragma unroll
      for (int j = 0; j < kRegSums; ++j) cs[j] += C[j];
    }
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) {
#pragma unroll
      for (int j = 0; j < kRegSums; ++j) cs[j] += __shfl_xor(cs[j], off, 64);
    }
    if ((tid & 63) == 0) {
#pragma unroll
      for (int j = 0; j < kRegSums; ++j) cred[tid >> 6][j] = cs[j];
    }
  }
  double s1 = 0.0, c1 = 0.0, s2 = 0.0, c2 = 0.0;
  unsigned long long kc[kItemCounters] = {0, 0, 0};
  for (int b0 = it0 + tid; b0 < it1; b0 += kFinishBatch * bs) {
    double4 P[kFinishBatch];
    unsigned long long K[kFinishBatch][kItemCounters];
#pragma unroll
    for (int u = 0; u < kFinishBatch; ++u) {
      const int it = b0 + u * bs;
      if (it < it1) {
        P[u] = reinterpret_cast<const double4 *>(a.partials)[it];
#pragma unroll
        for (int j = 0; j < kItemCounters; ++j)
          K[u][j] = a.counters[kItemCounters * static_cast<size_t>(it) + j];
      }
    }
#pragma unroll
    for (int u = 0; u < kFinishBatch; ++u) {
      if (b0 + u * bs < it1) {
        pair_merge(s1, c1, P[u].x, P[u].y);
        pair_merge(s2, c2, P[u].z, P[u].w);
#pragma unroll
        for (int j = 0; j < kItemCounters; ++j) kc[j] += K[u][j];
      }
    }
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
      const int slot = T->res_off + (T->it_done % T->res_cap);
      double *lg = a.reslog + 2 * slot;
      lg[0] = I;
      lg[1] = var;
      if (a.nreg > 0) {
        // components 1..nreg, then the extrapolation in the last pair
        double *cl = a.creslog + kRegSums * static_cast<size_t>(slot);
        for (int j = 0; j <= a.nreg; ++j) {
          const int r = j < a.nreg ? j : kMaxReg;
          double q1 = cred[0][2 * r], q2 = cred[0][2 * r + 1];
          for (int w = 1; w < (bs >> 6); ++w) {
            q1 += cred[w][2 * r];
            q2 += cred[w][2 * r + 1];
          }
          q1 /= N;
          q2 /= N;
          double v = (q2 - q1 * q1) / (N - 1.0);
          if (v < 0.0) v = 0.0;
          cl[2 * r] = T->shift + q1;
          cl[2 * r + 1] = v;
        }
      }
    }
    // training/evaluation split: the first evaluation iteration discards
    // the training iterations from the running sums
    if (T->train_iters > 0 && T->it_done == T->train_iters) {
      T->wsum = T->wisum = T->wi2sum = T->zsum = 0.0;
      T->nzero = 0;
      T->ncomb = 0;
    }
    T->ncomb += 1;
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
  // refinement: one wavefront per dimension; with a training phase the grid
  // is frozen once the training iterations are done
  __syncthreads();
  const int nb = a.phys.nb;
  const bool refine = T->train_iters <= 0 || T->it_done <= T->train_iters;
  double *scr = scratch + static_cast<size_t>(wave) * (2 * nb + 2);
  for (int m = wave; m < T->nd; m += (bs >> 6)) {
    double *hist = a.hists + T->hist_off + m * nb;
    double *edges = a.grids + T->grid_off + m * (nb + 1);
    if (refine) refine_dim_wave(hist, edges, nb, alpha, scr);
    __syncwarp();
    for (int b = lane; b < nb; b += 64) hist[b] = 0.0;
  }
}

// ---------------------------------------------------------------------------
// Hartree-Fock spectrum tables (eq:spe)

// Sigma_tau(k_i) [MeV] at the spline nodes k_i = i h of tasks [first,
// first + ntasks), one wavefront per (task, tau, node).  Over the occupied
// partners (isospin tau' < npartner, |k'| < kF_tau', every direction), with
// p = (k - k') / 2, the direct element V(p, p) counts for both partner spins
// and the exchange element V(p, -p) for equal spin and isospin:
//   Sigma_tau(k) = sum_tau' \int d^3k' / (2 pi)^3 [2 V(p, p) - delta_{tau tau'} V(p, -p)].
// Gauss-Legendre rule gl = (x[kHfGauss], w[kHfGauss]) on [-1, 1]: lane b takes
// the cosine node b and loops over the |k'| nodes; the azimuth gives 2 pi.
__global__ __launch_bounds__(256) void hf_nodes(KArgs a, const double *__restrict__ gl,
                                                int first, int ntasks, int ntab, int npartner) {
  const int wave = static_cast<int>((blockIdx.x * blockDim.x + threadIdx.x) >> 6);
  const int lane = threadIdx.x & 63;
  const int per_task = ntab * kHfEntries;
  if (wave >= ntasks * per_task) return;  // uniform per wavefront
  const int tl = wave / per_task, r = wave - tl * per_task;
  const int tau = r / kHfEntries, i = r - tau * kHfEntries;
  const TaskDev *__restrict__ T = a.tasks + first + tl;
  const double k = static_cast<double>(i) * T->hf_h;
  const Phys &ph = a.phys;
  const double vq0 = ph.V0 + ph.Vy / ph.m2;  // zero momentum transfer
  const double mu = gl[lane], wmu = gl[kHfGauss + lane];
  double acc = 0.0;
  for (int tp = 0; tp < npartner; ++tp) {
    const double kF = sqrt(T->kF2[tp]);
    if (!(kF > 0.0)) continue;
    double sum = 0.0;
    for (int j = 0; j < kHfGauss; ++j) {
      const double kp = 0.5 * kF * (gl[j] + 1.0), wk = 0.5 * kF * gl[kHfGauss + j];
      const double P2 = fmax(0.0, 0.25 * (k * k + kp * kp - 2.0 * k * kp * mu));
      double pn = P2;
      for (int e = 1; e < ph.half_exp; ++e) pn *= P2;
      const double reg = exp(-2.0 * pn * ph.invLn);
      double f = 2.0 * vq0;
      if (tp == tau) f -= ph.V0 + ph.Vy / (4.0 * P2 + ph.m2);
      sum = fma(wk * kp * kp, f * reg, sum);
    }
    acc = fma(wmu, sum, acc);
  }
  acc = wave_sum(acc) * (1.0 / (4.0 * M_PI * M_PI));  // 2 pi / (2 pi)^3
  if (lane == 0) a.hf[4 * static_cast<size_t>(T->hf_off + tau * kHfEntries + i)] = acc;
}

// Cubic spline with zero end slopes (Sigma is even in k and flat where the
// regulator has switched it off) through the node values of each (task, tau)
// table, one thread per table: second derivatives m from
//   2 m_0 + m_1 = 6 (y_1 - y_0) / h^2,
//   m_{i-1} + 4 m_i + m_{i+1} = 6 (y_{i+1} - 2 y_i + y_{i-1}) / h^2,
//   m_{n-1} + 2 m_n = -6 (y_n - y_{n-1}) / h^2
// (Thomas algorithm, the entries' spare slots as scratch), then per interval
// the coefficients of y_i + b t + c t^2 + d t^3, t = (k - k_i) / h.
__global__ void hf_spline(KArgs a, int first, int ntasks, int ntab) {
  const int id = static_cast<int>(blockIdx.x * blockDim.x + threadIdx.x);
  if (id >= ntasks * ntab) return;
  const int tl = id / ntab, tau = id - tl * ntab;
  const TaskDev *__restrict__ T = a.tasks + first + tl;
  double *E = a.hf + 4 * static_cast<size_t>(T->hf_off + tau * kHfEntries);
  constexpr int n = kHfIntervals;
  const double h2 = T->hf_h * T->hf_h;
  double bprev = 1.0, rprev = 0.0;
  for (int i = 0; i <= n; ++i) {
    double diag = (i == 0 || i == n) ? 2.0 : 4.0, r;
    if (i == 0) r = 6.0 * (E[4] - E[0]) / h2;
    else if (i == n) r = -6.0 * (E[4 * n] - E[4 * (n - 1)]) / h2;
    else r = 6.0 * (E[4 * (i + 1)] - 2.0 * E[4 * i] + E[4 * (i - 1)]) / h2;
    if (i > 0) {
      const double f = 1.0 / bprev;
      diag -= f;
      r -= f * rprev;
    }
    E[4 * i + 1] = diag;
    E[4 * i + 2] = r;
    bprev = diag;
    rprev = r;
  }
  double mnext = E[4 * n + 2] / E[4 * n + 1];
  E[4 * n + 3] = mnext;
  for (int i = n - 1; i >= 0; --i) {
    mnext = (E[4 * i + 2] - mnext) / E[4 * i + 1];
    E[4 * i + 3] = mnext;
  }
  for (int i = 0; i < n; ++i) {
    const double y0 = E[4 * i], y1 = E[4 * (i + 1)];
    const double m0 = E[4 * i + 3], m1 = E[4 * (i + 1) + 3];
    E[4 * i + 1] = (y1 - y0) - h2 * (2.0 * m0 + m1) / 6.0;
    E[4 * i + 2] = 0.5 * h2 * m0;
    E[4 * i + 3] = h2 * (m1 - m0) / 6.0;
  }
  E[4 * n + 1] = E[4 * n + 2] = E[4 * n + 3] = 0.0;
}

// Reset histograms and running state to zero, and the grids to uniform.
// keep_grid (a move to another EOS point): the grids and the Philox iteration
// word are kept, so the next iteration starts from the adapted grid with
// fresh random numbers, and only the new point's iterations enter the
// estimates.
__global__ void init_tasks(KArgs a, int first, int keep_grid) {
  TaskDev *T = a.tasks + first + blockIdx.x;
  const int nb = a.phys.nb;
  if (a.queue && blockIdx.x == 0 && threadIdx.x < kQueueSlots) a.queue[threadIdx.x] = 0;
  if (!keep_grid) {
    for (int i = threadIdx.x; i < T->nd * (nb + 1); i += blockDim.x) {
      const int b = i % (nb + 1);
      a.grids[T->grid_off + i] = static_cast<double>(b) / nb;
    }
  }
  for (int i = threadIdx.x; i < T->nd * nb; i += blockDim.x) a.hists[T->hist_off + i] = 0.0;
  if (threadIdx.x == 0) {
    if (!keep_grid) T->iter = 0;
    T->it_done = 0;
    T->shift = 0.0;
    T->wsum = T->wisum = T->wi2sum = T->zsum = 0.0;
    T->nzero = 0;
    T->ncomb = 0;
    T->lastI = T->lastV = 0.0;
    T->nevals = T->nfallback = T->npass = T->nterms = 0;
  }
}

// ---------------------------------------------------------------------------
// Host-side launchers

size_t sample_lds_bytes(int nd, int nb, int block, int ntab) {
  // turn and 2^(j/64) tables + HF tables + grid pairs + histogram + reduction
  // scratch + fp64 re-evaluation and Pauli screen queues (128 sample offsets
  // per wavefront each)
  return fixed_lds_bytes() + hf_lds_doubles(ntab) * sizeof(double) +
         (3 * static_cast<size_t>(nd) * nb + 6 * (block / 64)) * sizeof(double) +
         (block / 64) * 256 * sizeof(uint32_t);
}

// Dispatch on (order, q) to the launchers of kernels_inst.hip.
#define MBPT_OQ_SWITCH(CALL)                    \
  switch (order * 10 + q) {                     \
    case 12: return CALL(1, 2);                 \
    case 14: return CALL(1, 4);                 \
    case 22: return CALL(2, 2);                 \
    case 24: return CALL(2, 4);                 \
    case 32: return CALL(3, 2);                 \
    case 34: return CALL(3, 4);                 \
    case 42: return CALL(4, 2);                 \
    case 44: return CALL(4, 4);                 \
    case 52: return CALL(5, 2);                 \
    case 54: return CALL(5, 4);                 \
    default: return hipErrorInvalidValue;       \
  }

hipError_t launch_sample_single(const KArgs &a, int t, int order, int q, int prec, bool group,
                                int nitems, int block, hipStream_t st) {
#define MBPT_CALL(O, Q) launch_single_oq<O, Q>(a, t, prec, group, nitems, block, st)
  MBPT_OQ_SWITCH(MBPT_CALL)
#undef MBPT_CALL
}

hipError_t launch_sample_order(const KArgs &a, int order, int q, int prec, bool group, int k0,
                               int k1, int nitems, int block, hipStream_t st) {
#define MBPT_CALL(O, Q) launch_order_oq<O, Q>(a, prec, group, k0, k1, nitems, block, st)
  MBPT_OQ_SWITCH(MBPT_CALL)
#undef MBPT_CALL
}

hipError_t launch_sample_order_fixed4(const KArgs &a, int id, int prec, int k0, int k1, int nitems,
                                      int block, hipStream_t st) {
  switch (id / kFixed4Chunk) {
    case 0: return launch_o4_fixed<0>(a, id, prec, k0, k1, nitems, block, st);
    case 1: return launch_o4_fixed<10>(a, id, prec, k0, k1, nitems, block, st);
    case 2: return launch_o4_fixed<20>(a, id, prec, k0, k1, nitems, block, st);
    case 3: return launch_o4_fixed<30>(a, id, prec, k0, k1, nitems, block, st);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_sample_persistent(const KArgs &a, int order, int q, int prec, bool group, int k0,
                                    int k1, int nitems, int block, int cus, hipStream_t st) {
#define MBPT_CALL(O, Q) launch_persist_oq<O, Q>(a, prec, group, k0, k1, nitems, block, cus, st)
  MBPT_OQ_SWITCH(MBPT_CALL)
#undef MBPT_CALL
}

hipError_t launch_dump(const KArgs &a, int t, int order, int q, int prec, bool group,
                       uint32_t iter, uint64_t first, uint64_t count, double *out, double *out_reg,
                       hipStream_t st) {
#define MBPT_CALL(O, Q) launch_dump_oq<O, Q>(a, t, prec, group, iter, first, count, out, out_reg, st)
  MBPT_OQ_SWITCH(MBPT_CALL)
#undef MBPT_CALL
}

hipError_t launch_finish(const KArgs &a, int first_task, int ntasks, int step_iter, double alpha,
                         hipStream_t st) {
  const size_t lds =
      (kFinishThreads / 64) * static_cast<size_t>(2 * a.phys.nb + 2) * sizeof(double);
  hipLaunchKernelGGL(finish_iteration, dim3(ntasks), dim3(kFinishThreads), lds, st, a, first_task,
                     alpha, step_iter);
  return hipGetLastError();
}

hipError_t launch_hf(const KArgs &a, const double *gl, int first, int ntasks, int ntab,
                     int npartner, hipStream_t st) {
  const long waves = static_cast<long>(ntasks) * ntab * kHfEntries;
  hipLaunchKernelGGL(hf_nodes, dim3(static_cast<unsigned>((waves + 3) / 4)), dim3(256), 0, st, a,
                     gl, first, ntasks, ntab, npartner);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  const int threads = ntasks * ntab;
  hipLaunchKernelGGL(hf_spline, dim3((threads + 63) / 64), dim3(64), 0, st, a, first, ntasks, ntab);
  return hipGetLastError();
}

hipError_t launch_init(const KArgs &a, int first, int ntasks, hipStream_t st, bool keep_grid) {
  hipLaunchKernelGGL(init_tasks, dim3(ntasks), dim3(256), 0, st, a, first, keep_grid ? 1 : 0);
  return hipGetLastError();
}

}  // namespace mbpt
