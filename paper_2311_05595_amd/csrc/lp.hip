// The LP subproblem of the SLP step (Sec. 4.1, problem (Pstar)) for one linear
// constraint with a positive gradient (the volume):
//     min g^T s  s.t.  a^T s = b,  l <= s <= u,
//     l = max(-delta, x_l - x),  u = min(delta, x_u - x).
// From s = l the variables are raised in order of the ratio r = -g / a
// (highest first, equal ratios in index order), each to u, until the volume
// budget B = b - a^T l is used; the variable that reaches it is raised
// partially, and its ratio is the multiplier of the constraint.
//
// The order is never sorted globally.  The critical ratio is found by a radix
// select over 64-bit keys that order the ratios from high to low: eight
// passes of eight bits.  Each pass builds per-block sums of the capacities
// a (u - l) per key digit: a block loads chunks of 256 items, sorts each chunk
// by digit in LDS (ranks from ballots of the digit's bits, slots from a scan
// of per-wave counts), and sums each digit's run with a segmented scan inside
// each wave, so every sum is taken in a fixed order.  The sums are reduced in
// a fixed order and the pass picks the digit where the running capacity
// reaches the remaining budget.  Variables above the critical key go to u,
// below to l; the tied group at the key shares what is left of the budget in
// index order through a block-wise scan.  A feasibility flag in the device
// state selects, without a host round trip, between that solution and the
// box end of the artificial problem (Sec. 4.2) when the budget lies outside
// the box's range.
#include <cmath>
#include <cstring>
#include <string>

#include "lp.h"

namespace mgcg {

namespace {

constexpr int LP_BS = 256;    // threads per block; also items per block
constexpr int LP_ROWS = 64;   // partial-bin rows summed per block of the first reduction
constexpr int LP_SUM_BLOCKS = 1024;
constexpr int LP_CH = 8;             // most chunks of LP_BS items per block of the digit passes  // blocks of the grid-stride sums of the thresholding

struct LpState {
  unsigned long long prefix;  // key digits picked so far (high bits)
  double remaining;           // budget still to place within the prefix's items
  double budget, capsum;      // B (clamped to [0, capsum] when feasible) and the total capacity
  int bad;                    // a non-positive or non-finite a, or non-finite g, x
  int feasible;               // B within [0, capsum] up to the rounding of its sums
};

__device__ __forceinline__ unsigned long long ratio_key(double r) {
  if (r == 0.0) r = 0.0;  // one key for +0 and -0
  unsigned long long u = (unsigned long long)__double_as_longlong(r);
  u = (u >> 63) ? ~u : (u | 0x8000000000000000ull);  // ascending with r
  return ~u;                                         // ascending key = descending ratio
}
__device__ __forceinline__ double key_ratio(unsigned long long k) {
  unsigned long long u = ~k;
  u = (u >> 63) ? (u & 0x7FFFFFFFFFFFFFFFull) : ~u;
  return __longlong_as_double((long long)u);
}

// Fixed-order sum of one value per thread (thread 0 gets it).
__device__ __forceinline__ double block_sum_lp(double v, double* sh) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) sh[w] = v;
  __syncthreads();
  double t = 0.0;
  if (threadIdx.x == 0)
    for (int i = 0; i < LP_BS / 64; ++i) t += sh[i];
  return t;
}

__global__ __launch_bounds__(LP_BS) void k_lp_prep(long n, const double* __restrict__ g,
                                                   const double* __restrict__ a,
                                                   const double* __restrict__ x, double delta,
                                                   double xl, double xu,
                                                   const unsigned char* __restrict__ fixed,
                                                   unsigned long long* __restrict__ key,
                                                   double* __restrict__ cap,
                                                   double* __restrict__ part, LpState* st) {
  __shared__ double sh[LP_BS / 64];
  const long i = (long)blockIdx.x * LP_BS + threadIdx.x;
  double al = 0.0, c = 0.0, aal = 0.0;
  if (i < n) {
    const double gi = g[i], ai = a[i], xi = x[i];
    const bool fx = fixed && fixed[i];
    const double l = fx ? 0.0 : fmax(-delta, xl - xi), u = fx ? 0.0 : fmin(delta, xu - xi);
    const bool ok = ai > 0.0 && isfinite(ai) && isfinite(gi) && isfinite(xi) && l <= u;
    if (!ok) st->bad = 1;
    c = ok ? ai * (u - l) : 0.0;
    al = ok ? ai * l : 0.0;
    aal = fabs(al);
    key[i] = ratio_key(ok ? -gi / ai : 0.0);
    cap[i] = c;
  }
  const double s0 = block_sum_lp(al, sh);
  const double s1 = block_sum_lp(c, sh);
  const double s2 = block_sum_lp(aal, sh);
  if (threadIdx.x == 0) {
    part[blockIdx.x] = s0;
    part[gridDim.x + blockIdx.x] = s1;
    part[2 * gridDim.x + blockIdx.x] = s2;
  }
}

// B = b - a^T l and the total capacity, summed in block order.  A budget
// within the rounding allowance 2 n eps (sum |a l| + capacity) of 0 or of the
// capacity is the boundary itself (clamped); beyond it the LP has no solution.
__global__ __launch_bounds__(LP_BS) void k_lp_budget(long n, int nb, double b,
                                                     const double* __restrict__ part, LpState* st) {
  __shared__ double sh[LP_BS / 64];
  double s0 = 0.0, s1 = 0.0, s2 = 0.0;
  for (int j = threadIdx.x; j < nb; j += LP_BS) {
    s0 += part[j];
    s1 += part[nb + j];
    s2 += part[2 * nb + j];
  }
  const double al = block_sum_lp(s0, sh);
  const double cs = block_sum_lp(s1, sh);
  const double aal = block_sum_lp(s2, sh);
  if (threadIdx.x == 0) {
    const double B = b - al;
    const double tau = 2.0 * (double)n * 2.220446049250313e-16 * (aal + cs);
    const int ok = B >= -tau && B <= cs + tau;
    const double Bc = fmin(fmax(B, 0.0), cs);
    st->budget = ok ? Bc : B;
    st->capsum = cs;
    st->remaining = Bc;
    st->feasible = ok;
    st->prefix = 0ull;
  }
}

// Pass over digit d (bits 63 - 8d .. 56 - 8d): per block of ch (<= LP_CH)
// consecutive chunks of LP_BS items, the capacity sum of the items whose
// higher digits equal the prefix, per value of digit d, in a fixed order.
// The keys (and capacities) of all chunks are loaded first.  Each chunk is then
// sorted by digit in LDS, stably: the lanes of a wave with the same digit come
// from eight ballots of the digit's bits, their rank is the count of such
// lanes below, and a block-wide scan of the per-wave counts gives each digit's
// first slot.  A segmented scan within each wave sums the runs of equal digits;
// thread t adds the (at most four) wave pieces of digit t's run, chunk after
// chunk.  UNIT: every capacity is 1 (not read).
template <bool UNIT>
__global__ __launch_bounds__(LP_BS) void k_lp_hist(long n, int d, int ch,
                                                   const unsigned long long* __restrict__ key,
                                                   const double* __restrict__ cap,
                                                   const LpState* st, double* __restrict__ bins) {
  static_assert(LP_BS == 256, "one thread per digit value");
  if (!st->feasible) return;  // the artificial problem's box end instead
  __shared__ int pos[LP_BS / 64][256];  // per wave: count of each digit, then its first slot
  __shared__ int wtot[LP_BS / 64];
  __shared__ int first_s[256];          // first slot of each digit
  __shared__ int sdig[LP_BS];           // digit of each slot
  __shared__ double sval[LP_BS];        // capacity of each slot, then the run's running sum
  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
  const unsigned long long pre = st->prefix;
  const int shift = 56 - 8 * d;
  const unsigned long long lower = (1ull << lane) - 1ull;
  const long base = (long)blockIdx.x * ch * LP_BS + t;
  unsigned long long kk[LP_CH];
  bool mm[LP_CH];
  double cc[LP_CH];
#pragma unroll
  for (int c = 0; c < LP_CH; ++c) {
    const long i = base + (long)c * LP_BS;
    kk[c] = (c < ch && i < n) ? key[i] : 0ull;
  }
#pragma unroll
  for (int c = 0; c < LP_CH; ++c) {
    const long i = base + (long)c * LP_BS;
    mm[c] = c < ch && i < n && (d == 0 || (kk[c] >> (shift + 8)) == (pre >> (shift + 8)));
    cc[c] = UNIT ? 1.0 : (mm[c] ? cap[i] : 0.0);
  }
  if (UNIT) {
    // unit capacities: the sums are counts, exact in any order; one LDS
    // atomic per run of equal digits in a wave
    __shared__ int hcount[256];
    hcount[t] = 0;
    __syncthreads();
#pragma unroll
    for (int c = 0; c < LP_CH; ++c) {
      if (c >= ch) break;
      const bool match = mm[c];
      const int dig = (int)((kk[c] >> shift) & 255ull);
      unsigned long long same = __ballot(match);
#pragma unroll
      for (int bit = 0; bit < 8; ++bit) {
        const int on = (dig >> bit) & 1;
        const unsigned long long m = __ballot(on);
        same &= on ? m : ~m;
      }
      if (match && (same & lower) == 0ull) atomicAdd(&hcount[dig], __popcll(same));
    }
    __syncthreads();
    bins[(long)blockIdx.x * 256 + t] = (double)hcount[t];
    return;
  }
  double s = 0.0;
#pragma unroll
  for (int c = 0; c < LP_CH; ++c) {
    if (c >= ch) break;
    const bool match = mm[c];
    // a chunk with no item inside the prefix adds nothing (block-uniform)
    if (!__syncthreads_or(match)) continue;
    const int dig = (int)((kk[c] >> shift) & 255ull);
#pragma unroll
    for (int q = 0; q < LP_BS / 64; ++q) pos[q][t] = 0;
    unsigned long long same = __ballot(match);
#pragma unroll
    for (int bit = 0; bit < 8; ++bit) {
      const int on = (dig >> bit) & 1;
      const unsigned long long m = __ballot(on);
      same &= on ? m : ~m;
    }
    const int rank = __popcll(same & lower);
    __syncthreads();
    if (match && rank == 0) pos[w][dig] = __popcll(same);
    __syncthreads();
    int cnt[LP_BS / 64], tot = 0;
#pragma unroll
    for (int q = 0; q < LP_BS / 64; ++q) {
      cnt[q] = pos[q][t];
      tot += cnt[q];
    }
    int incl = tot;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
      const int o = __shfl_up(incl, off, 64);
      if (lane >= off) incl += o;
    }
    if (lane == 63) wtot[w] = incl;
    __syncthreads();
    int first = incl - tot, total = 0;
#pragma unroll
    for (int q = 0; q < LP_BS / 64; ++q) {
      if (q < w) first += wtot[q];
      total += wtot[q];
    }
    first_s[t] = first;
    int run = first;
#pragma unroll
    for (int q = 0; q < LP_BS / 64; ++q) {
      pos[q][t] = run;
      run += cnt[q];
    }
    __syncthreads();
    if (match) {
      const int slot = pos[w][dig] + rank;
      sval[slot] = cc[c];
      sdig[slot] = dig;
    }
    __syncthreads();
    // segmented inclusive scan of the slots within each wave (runs of one digit)
    double v = 0.0;
    int seg0 = 64;
    if (t < total) {
      v = sval[t];
      const int f = first_s[sdig[t]] - 64 * w;
      seg0 = f > 0 ? f : 0;
    }
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
      const double o = __shfl_up(v, off, 64);
      if (lane - off >= seg0) v += o;
    }
    sval[t] = v;
    __syncthreads();
    if (tot > 0) {
      const int end = first + tot;
      for (int q = first >> 6; q <= (end - 1) >> 6; ++q) {
        const int last = end < 64 * q + 64 ? end : 64 * q + 64;
        s += sval[last - 1];
      }
    }
    __syncthreads();
  }
  bins[(long)blockIdx.x * 256 + t] = s;
}

// Rows [LP_ROWS j, LP_ROWS (j + 1)) of the per-block bins summed per digit.
__global__ __launch_bounds__(LP_BS) void k_lp_reduce(int nb, const double* __restrict__ bins,
                                                     double* __restrict__ out, const LpState* st) {
  if (!st->feasible) return;
  const int r0 = blockIdx.x * LP_ROWS;
  const int r1 = min(r0 + LP_ROWS, nb);
  double s = 0.0;
  // loads of 16 rows in flight, summed in row order
  for (int r = r0; r < r1; r += 16) {
    double v[16];
#pragma unroll
    for (int q = 0; q < 16; ++q) v[q] = r + q < r1 ? bins[(long)(r + q) * 256 + threadIdx.x] : 0.0;
#pragma unroll
    for (int q = 0; q < 16; ++q) s += v[q];
  }
  out[(long)blockIdx.x * 256 + threadIdx.x] = s;
}

// Digit d of the critical key: the first digit (ascending key, i.e. highest
// ratios first) whose running capacity reaches the remaining budget.
__global__ __launch_bounds__(LP_BS) void k_lp_pick(int nrows, int d, const double* __restrict__ part,
                                                   LpState* st) {
  if (!st->feasible) return;
  __shared__ double wtot[LP_BS / 64];
  __shared__ int first[LP_BS / 64], lastb[LP_BS / 64];
  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
  // this digit's capacity, the rows summed in order with their loads in flight
  double tot = 0.0;
  for (int r = 0; r < nrows; r += 16) {
    double v[16];
#pragma unroll
    for (int q = 0; q < 16; ++q) v[q] = r + q < nrows ? part[(long)(r + q) * 256 + t] : 0.0;
#pragma unroll
    for (int q = 0; q < 16; ++q) tot += v[q];
  }
  // running capacity before this digit (ascending digits): a scan within the
  // wave, then the totals of the waves before it
  double incl = tot;
#pragma unroll
  for (int off = 1; off < 64; off <<= 1) {
    const double o = __shfl_up(incl, off, 64);
    if (lane >= off) incl += o;
  }
  if (lane == 63) wtot[w] = incl;
  __syncthreads();
  double before = incl - tot;
  for (int j = 0; j < w; ++j) before += wtot[j];
  const double rem = st->remaining;
  // the first digit with capacity whose running capacity reaches rem, and the
  // last digit with capacity (the fallback when rounding leaves none)
  const bool hit = tot > 0.0 && before + tot >= rem;
  int f = hit ? t : 1 << 30, l = tot > 0.0 ? t : -1;
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    f = min(f, __shfl_down(f, off, 64));
    l = max(l, __shfl_down(l, off, 64));
  }
  if (lane == 0) {
    first[w] = f;
    lastb[w] = l;
  }
  __syncthreads();
  int pick = 1 << 30, last = -1;
  for (int j = 0; j < LP_BS / 64; ++j) {
    pick = min(pick, first[j]);
    last = max(last, lastb[j]);
  }
  const bool fallback = pick == (1 << 30);
  if (fallback) pick = last < 0 ? 0 : last;
  __syncthreads();
  if (t == pick) {
    st->remaining = (fallback && last < 0) ? rem : rem - before;
    st->prefix |= (unsigned long long)pick << (56 - 8 * d);
  }
}

// Capacity of the tied items (key == the critical key) per block.
template <bool UNIT>
__global__ __launch_bounds__(LP_BS) void k_lp_tiesum(long n, const unsigned long long* __restrict__ key,
                                                     const double* __restrict__ cap,
                                                     const LpState* st, double* __restrict__ tsum) {
  if (!st->feasible) return;
  __shared__ double sh[LP_BS / 64];
  const long i = (long)blockIdx.x * LP_BS + threadIdx.x;
  const unsigned long long T = st->prefix;
  const double c = (i < n && key[i] == T) ? (UNIT ? 1.0 : cap[i]) : 0.0;
  const double s = block_sum_lp(c, sh);
  if (threadIdx.x == 0) tsum[blockIdx.x] = s;
}

// Exclusive scan of the per-block tied capacities (one block, in order): tiles
// of LP_BS * 8 entries staged in LDS with coalesced loads, each thread's eight
// consecutive entries summed, a block scan of those sums, the tile's total
// carried to the next tile.
__global__ __launch_bounds__(LP_BS) void k_lp_tiescan(int nb, double* __restrict__ tsum,
                                                      const LpState* st) {
  if (st && !st->feasible) return;
  constexpr int PER = 8, TILE = LP_BS * PER;
  __shared__ double tile[TILE];
  __shared__ double wt[LP_BS / 64];
  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
  double carry = 0.0;
  for (int base = 0; base < nb; base += TILE) {
#pragma unroll
    for (int q = 0; q < PER; ++q) {
      const int j = base + q * LP_BS + t;
      tile[q * LP_BS + t] = j < nb ? tsum[j] : 0.0;
    }
    __syncthreads();
    double v[PER], sum = 0.0;
#pragma unroll
    for (int q = 0; q < PER; ++q) {
      v[q] = tile[t * PER + q];
      sum += v[q];
    }
    double incl = sum;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
      const double o = __shfl_up(incl, off, 64);
      if (lane >= off) incl += o;
    }
    double excl = __shfl_up(incl, 1, 64);
    if (lane == 0) excl = 0.0;
    if (lane == 63) wt[w] = incl;
    __syncthreads();
    double pre = carry, tile_total = 0.0;
#pragma unroll
    for (int q = 0; q < LP_BS / 64; ++q) {
      if (q < w) pre += wt[q];
      tile_total += wt[q];
    }
    pre += excl;
#pragma unroll
    for (int q = 0; q < PER; ++q) {
      tile[t * PER + q] = pre;
      pre += v[q];
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < PER; ++q) {
      const int j = base + q * LP_BS + t;
      if (j < nb) tsum[j] = tile[q * LP_BS + t];
    }
    carry += tile_total;
    __syncthreads();
  }
}

// s from the critical key: u above it, l below it, the tied items in index
// order up to the remaining budget; block partials of g^T s, a^T s, |s|_inf.
__global__ __launch_bounds__(LP_BS) void k_lp_fill(long n, const double* __restrict__ g,
                                                   const double* __restrict__ a,
                                                   const double* __restrict__ x, double delta,
                                                   double xl, double xu,
                                                   const unsigned char* __restrict__ fixed,
                                                   const unsigned long long* __restrict__ key,
                                                   const double* __restrict__ cap,
                                                   const double* __restrict__ toff,
                                                   const LpState* st, double* __restrict__ s,
                                                   double* __restrict__ part) {
  if (!st->feasible) return;
  __shared__ double sh[LP_BS / 64];
  __shared__ double wsum[LP_BS / 64];
  const long i = (long)blockIdx.x * LP_BS + threadIdx.x;
  const unsigned long long T = st->prefix;
  const double R = st->remaining;
  double gi = 0.0, ai = 0.0, l = 0.0, u = 0.0, c = 0.0;
  unsigned long long k = ~0ull;
  if (i < n) {
    gi = g[i];
    ai = a[i];
    const double xi = x[i];
    const bool fx = fixed && fixed[i];
    l = fx ? 0.0 : fmax(-delta, xl - xi);
    u = fx ? 0.0 : fmin(delta, xu - xi);
    k = key[i];
    c = cap[i];
  }
  // exclusive scan of the tied capacities in index order within the block
  const double tc = (i < n && k == T) ? c : 0.0;
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  double incl = tc;
#pragma unroll
  for (int off = 1; off < 64; off <<= 1) {
    const double o = __shfl_up(incl, off, 64);
    if (lane >= off) incl += o;
  }
  if (lane == 63) wsum[w] = incl;
  __syncthreads();
  double before = toff[blockIdx.x];
  for (int j = 0; j < w; ++j) before += wsum[j];
  before += incl - tc;
  double si = 0.0;
  if (i < n) {
    if (k < T) {
      si = u;
    } else if (k > T) {
      si = l;
    } else {
      const double take = fmin(c, fmax(0.0, R - before));
      si = take >= c ? u : l + take / ai;
    }
    s[i] = si;
  }
  const double p0 = block_sum_lp(gi * si, sh);
  const double p1 = block_sum_lp(ai * si, sh);
  double m = fabs(si);
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) m = fmax(m, __shfl_down(m, off, 64));
  __syncthreads();
  if (lane == 0) sh[w] = m;
  __syncthreads();
  if (threadIdx.x == 0) {
    double mm = 0.0;
    for (int j = 0; j < LP_BS / 64; ++j) mm = fmax(mm, sh[j]);
    part[blockIdx.x] = p0;
    part[gridDim.x + blockIdx.x] = p1;
    part[2 * gridDim.x + blockIdx.x] = mm;
  }
}

// The shrunk box end of the artificial problem (Sec. 4.1.2): s = l' (upper
// false) or u' (upper true) with the radius 0.8 delta.
__global__ __launch_bounds__(LP_BS) void k_lp_box(long n, const double* __restrict__ g,
                                                  const double* __restrict__ a,
                                                  const double* __restrict__ x, double delta,
                                                  double xl, double xu,
                                                  const unsigned char* __restrict__ fixed,
                                                  const LpState* st, double* __restrict__ s,
                                                  double* __restrict__ part) {
  if (st->feasible) return;  // the LP's own solution instead
  const int upper = st->budget > st->capsum;
  __shared__ double sh[LP_BS / 64];
  const long i = (long)blockIdx.x * LP_BS + threadIdx.x;
  double gi = 0.0, ai = 0.0, si = 0.0;
  if (i < n) {
    gi = g[i];
    ai = a[i];
    const double xi = x[i];
    si = (fixed && fixed[i]) ? 0.0
                             : (upper ? fmin(0.8 * delta, xu - xi) : fmax(-0.8 * delta, xl - xi));
    s[i] = si;
  }
  const double p0 = block_sum_lp(gi * si, sh);
  const double p1 = block_sum_lp(ai * si, sh);
  double m = fabs(si);
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) m = fmax(m, __shfl_down(m, off, 64));
  __syncthreads();
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  if (lane == 0) sh[w] = m;
  __syncthreads();
  if (threadIdx.x == 0) {
    double mm = 0.0;
    for (int j = 0; j < LP_BS / 64; ++j) mm = fmax(mm, sh[j]);
    part[blockIdx.x] = p0;
    part[gridDim.x + blockIdx.x] = p1;
    part[2 * gridDim.x + blockIdx.x] = mm;
  }
}

// g^T s, a^T s and |s|_inf from the block partials, in block order.
__global__ __launch_bounds__(LP_BS) void k_lp_info(int nb, const double* __restrict__ part,
                                                   double* __restrict__ out) {
  __shared__ double sh[LP_BS / 64];
  double s0 = 0.0, s1 = 0.0, m = 0.0;
  for (int j = threadIdx.x; j < nb; j += LP_BS) {
    s0 += part[j];
    s1 += part[nb + j];
    m = fmax(m, part[2 * nb + j]);
  }
  const double gts = block_sum_lp(s0, sh);
  const double ats = block_sum_lp(s1, sh);
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) m = fmax(m, __shfl_down(m, off, 64));
  __syncthreads();
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  if (lane == 0) sh[w] = m;
  __syncthreads();
  if (threadIdx.x == 0) {
    double mm = 0.0;
    for (int j = 0; j < LP_BS / 64; ++j) mm = fmax(mm, sh[j]);
    out[0] = gts;
    out[1] = ats;
    out[2] = mm;
  }
}

// ---- thresholding of Sec. 5 on the same scratch

// Keys of the values (descending); the capacities are 1 (never stored): the
// radix select then picks the k-th largest value, equal values in index order.
__global__ __launch_bounds__(LP_BS) void k_sel_prep(long n, const double* __restrict__ v,
                                                    unsigned long long* __restrict__ key,
                                                    LpState* st) {
  const long i = (long)blockIdx.x * LP_BS + threadIdx.x;
  if (i < n) {
    const double vi = v[i];
    if (!isfinite(vi)) st->bad = 1;
    key[i] = ratio_key(isfinite(vi) ? vi : 0.0);
  }
}
__global__ void k_sel_budget(double k, LpState* st) {
  if (threadIdx.x == 0) {
    st->remaining = k;
    st->budget = k;
    st->prefix = 0ull;
    st->feasible = 1;
  }
}
// 1 for the k largest values (keys below the critical key, and the first
// ones of the tied group in index order), 0 for the rest.
__global__ __launch_bounds__(LP_BS) void k_sel_fill(long n, const unsigned long long* __restrict__ key,
                                                    const double* __restrict__ toff,
                                                    const LpState* st, double* __restrict__ out) {
  __shared__ double wsum[LP_BS / 64];
  const long i = (long)blockIdx.x * LP_BS + threadIdx.x;
  const unsigned long long T = st->prefix;
  const double R = st->remaining;
  const unsigned long long k = i < n ? key[i] : ~0ull;
  const double tc = (i < n && k == T) ? 1.0 : 0.0;
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  double incl = tc;
#pragma unroll
  for (int off = 1; off < 64; off <<= 1) {
    const double o = __shfl_up(incl, off, 64);
    if (lane >= off) incl += o;
  }
  if (lane == 63) wsum[w] = incl;
  __syncthreads();
  double before = toff[blockIdx.x];
  for (int j = 0; j < w; ++j) before += wsum[j];
  before += incl - tc;
  if (i < n) out[i] = k < T ? 1.0 : (k > T ? 0.0 : (R - before >= 1.0 ? 1.0 : 0.0));
}

// Rounding of the densities very close to 0 or 1.
// (out may be r: each item is read, then written, by one thread)
__global__ __launch_bounds__(LP_BS) void k_round(long n, const double* r, double lo, double hi,
                                                 double* out) {
  const long i = (long)blockIdx.x * LP_BS + threadIdx.x;
  if (i < n) {
    const double v = r[i];
    out[i] = v >= hi ? 1.0 : (v <= lo ? 0.0 : v);
  }
}

// Block partials of three sums: a^T b, a^T a, b^T b (grid-stride: each thread
// adds its items in a fixed order).
__global__ __launch_bounds__(LP_BS) void k_dot3(long n, const double* __restrict__ a,
                                                const double* __restrict__ b,
                                                double* __restrict__ part) {
  __shared__ double sh[LP_BS / 64];
  double s0 = 0.0, s1 = 0.0, s2 = 0.0;
  const long stride = (long)gridDim.x * LP_BS;
  for (long i = (long)blockIdx.x * LP_BS + threadIdx.x; i < n; i += stride) {
    const double x = a[i], y = b[i];
    s0 += x * y;
    s1 += x * x;
    s2 += y * y;
  }
  s0 = block_sum_lp(s0, sh);
  s1 = block_sum_lp(s1, sh);
  s2 = block_sum_lp(s2, sh);
  if (threadIdx.x == 0) {
    part[blockIdx.x] = s0;
    part[gridDim.x + blockIdx.x] = s1;
    part[2 * gridDim.x + blockIdx.x] = s2;
  }
}
// The three sums from the block partials, in block order.
__global__ __launch_bounds__(LP_BS) void k_sum3(int nb, const double* __restrict__ part,
                                                double* __restrict__ out) {
  __shared__ double sh[LP_BS / 64];
  double s[3] = {0.0, 0.0, 0.0};
  for (int j = threadIdx.x; j < nb; j += LP_BS)
    for (int q = 0; q < 3; ++q) s[q] += part[q * nb + j];
  for (int q = 0; q < 3; ++q) {
    const double t = block_sum_lp(s[q], sh);
    if (threadIdx.x == 0) out[q] = t;
  }
}

// Smooth Heaviside projection (Sec. 5.4):
//   h = (tanh(beta eta) + tanh(beta (rho - eta))) / (tanh(beta eta) + tanh(beta (1 - eta)))
// and its derivative in eta; per block the partial sums of h, dh/deta and rho
// (Newton's method on the volume runs on the host).
// h and dh/deta at one density; inv = 1 / (tanh(beta eta) + tanh(beta (1 - eta)))
// (the sums of Newton's method multiply by it; the projected values divide).
__device__ __forceinline__ void heaviside_at(double r, double beta, double eta, double te,
                                             double t1, double inv, double& h, double& dh) {
  const double tr = tanh(beta * (r - eta));
  const double num = te + tr, den = te + t1;
  const double dnum = beta * (1.0 - te * te) - beta * (1.0 - tr * tr);
  const double dden = beta * (1.0 - te * te) - beta * (1.0 - t1 * t1);
  h = num * inv;
  dh = (dnum * den - num * dden) * (inv * inv);
}
__global__ __launch_bounds__(LP_BS) void k_hv_sums(long n, const double* __restrict__ r, double beta,
                                                   double eta, double* __restrict__ part) {
  __shared__ double sh[LP_BS / 64];
  const double te = tanh(beta * eta), t1 = tanh(beta * (1.0 - eta));
  const double inv = 1.0 / (te + t1);
  double s0 = 0.0, s1 = 0.0, s2 = 0.0;
  const long stride = (long)gridDim.x * LP_BS;
  for (long i = (long)blockIdx.x * LP_BS + threadIdx.x; i < n; i += stride) {
    const double ri = r[i];
    double h, dh;
    heaviside_at(ri, beta, eta, te, t1, inv, h, dh);
    s0 += h;
    s1 += dh;
    s2 += ri;
  }
  s0 = block_sum_lp(s0, sh);
  s1 = block_sum_lp(s1, sh);
  s2 = block_sum_lp(s2, sh);
  if (threadIdx.x == 0) {
    part[blockIdx.x] = s0;
    part[gridDim.x + blockIdx.x] = s1;
    part[2 * gridDim.x + blockIdx.x] = s2;
  }
}
__global__ __launch_bounds__(LP_BS) void k_hv_apply(long n, const double* __restrict__ r, double beta,
                                                    double eta, double* __restrict__ out) {
  const double te = tanh(beta * eta), t1 = tanh(beta * (1.0 - eta));
  const double den = te + t1;
  const long stride = (long)gridDim.x * LP_BS;
  for (long i = (long)blockIdx.x * LP_BS + threadIdx.x; i < n; i += stride)
    out[i] = (te + tanh(beta * (r[i] - eta))) / den;
}


// ---- the strategy based on the gradient of the Lagrangian (Sec. 5.2)
//
// alpha_i: the step at which rho_i - alpha g_i reaches 0 (g_i > 0) or 1
// (g_i < 0); inf for g_i = 0.  With m_i = min(alpha, alpha_i) the step's
// cosine with -g is sum g^2 m / (|g| sqrt(sum g^2 m^2)), nonincreasing in
// alpha, so the admissible steps form an interval: the largest alpha (as a
// double) below the first safeguard violation whose cosine passes is found
// by a 16-way search over the bits of alpha (16 passes of two sums at 15
// points each), and alpha~ is the largest alpha_i > 0 up to it.

struct LgState {
  unsigned long long lo, hi;  // search bracket (bits of non-negative doubles): lo passes, hi not
  double viol;                // smallest alpha_i of a density the safeguards forbid to round
  double wsum;                // |g|^2
  double amax;                // largest finite alpha_i
  double alpha;               // alpha~
  // after the compaction: the sums of the items below the bracket
  // (sum g^2 alpha, sum g^2 alpha^2), the weight above it (sum g^2) and the
  // number of items inside it, which alone are read from then on
  double c1, c2, whi;
  double mid;
};
static_assert(sizeof(LgState) <= 256, "the state shares the LP state's slot");
constexpr int LG_PTS = 15;    // interior points of the search per pass
constexpr int LG_FULL = 4;    // passes over every item before the compaction

__device__ __forceinline__ double lg_alpha(double r, double g) {
  return g > 0.0 ? r / g : (g < 0.0 ? (1.0 - r) / -g : INFINITY);
}

__device__ __forceinline__ double block_min_lp(double v, double* sh) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v = fmin(v, __shfl_down(v, off, 64));
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) sh[w] = v;
  __syncthreads();
  double t = INFINITY;
  if (threadIdx.x == 0)
    for (int i = 0; i < LP_BS / 64; ++i) t = fmin(t, sh[i]);
  return t;
}
__device__ __forceinline__ double block_max_lp(double v, double* sh) {
  return -block_min_lp(-v, sh);
}

// alpha, g^2 and block partials of the violation minimum, |g|^2 and max alpha.
__global__ __launch_bounds__(LP_BS) void k_lg_prep(long n, const double* __restrict__ rho,
                                                   const double* __restrict__ g, double vu,
                                                   double vl, double* __restrict__ alpha,
                                                   double* __restrict__ w,
                                                   double* __restrict__ part, LpState* st) {
  __shared__ double sh[LP_BS / 64];
  double vmin = INFINITY, ws = 0.0, am = 0.0;
  const long stride = (long)gridDim.x * LP_BS;
  for (long i = (long)blockIdx.x * LP_BS + threadIdx.x; i < n; i += stride) {
    const double r = rho[i], gi = g[i];
    if (!isfinite(r) || !isfinite(gi)) st->bad = 1;
    const double a = lg_alpha(r, gi);
    alpha[i] = a;
    w[i] = gi * gi;
    ws += gi * gi;
    if ((gi < 0.0 && r < vu) || (gi > 0.0 && r > vl)) vmin = fmin(vmin, a);
    if (isfinite(a)) am = fmax(am, a);
  }
  vmin = block_min_lp(vmin, sh);
  ws = block_sum_lp(ws, sh);
  am = block_max_lp(am, sh);
  if (threadIdx.x == 0) {
    part[blockIdx.x] = vmin;
    part[gridDim.x + blockIdx.x] = ws;
    part[2 * gridDim.x + blockIdx.x] = am;
  }
}

__global__ __launch_bounds__(LP_BS) void k_lg_init(int nb, const double* __restrict__ part,
                                                   LgState* st) {
  __shared__ double sh[LP_BS / 64];
  double vmin = INFINITY, ws = 0.0, am = 0.0;
  for (int j = threadIdx.x; j < nb; j += LP_BS) {
    vmin = fmin(vmin, part[j]);
    ws += part[nb + j];
    am = fmax(am, part[2 * nb + j]);
  }
  vmin = block_min_lp(vmin, sh);
  ws = block_sum_lp(ws, sh);
  am = block_max_lp(am, sh);
  if (threadIdx.x == 0) {
    st->viol = vmin;
    st->wsum = ws;
    st->amax = am;
    st->alpha = 0.0;
    st->c1 = 0.0;
    st->c2 = 0.0;
    st->whi = 0.0;
    st->mid = 0.0;
    st->lo = 0ull;
    // every alpha_i beyond amax gives the cosine at amax: search [0, nextafter(amax))
    const double cap = fmin(vmin, nextafter(am, INFINITY));
    st->hi = am > 0.0 ? (unsigned long long)__double_as_longlong(cap) : 0ull;
  }
}

__device__ __forceinline__ double lg_point(unsigned long long lo, unsigned long long hi, int p) {
  const unsigned long long d = hi - lo;
  const unsigned long long x = lo + (d >> 4) * (unsigned long long)p + (((d & 15ull) * p) >> 4);
  return __longlong_as_double((long long)x);
}

// Block partials of sum g^2 m and sum g^2 m^2 at the LG_PTS interior points.
__global__ __launch_bounds__(LP_BS) void k_lg_split(long n, const double* __restrict__ alpha,
                                                    const double* __restrict__ w, int step,
                                                    const LgState* st, double* __restrict__ part) {
  __shared__ double sh[LP_BS / 64][2 * LG_PTS];
  const unsigned long long lo = st->lo, hi = st->hi;
  double x[LG_PTS], s1[LG_PTS], s2[LG_PTS];
#pragma unroll
  for (int p = 0; p < LG_PTS; ++p) {
    x[p] = lg_point(lo, hi, p + 1);
    s1[p] = 0.0;
    s2[p] = 0.0;
  }
  const long stride = (long)gridDim.x * LP_BS;
  if (hi - lo > 1ull) {
    for (long i = (long)blockIdx.x * LP_BS + threadIdx.x; i < n; i += stride) {
      const double a = alpha[i * step], wi = w[i * step];
#pragma unroll
      for (int p = 0; p < LG_PTS; ++p) {
        const double m = fmin(x[p], a);
        const double wm = wi * m;
        s1[p] += wm;
        s2[p] += wm * m;
      }
    }
  }
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
  for (int p = 0; p < LG_PTS; ++p) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
      s1[p] += __shfl_down(s1[p], off, 64);
      s2[p] += __shfl_down(s2[p], off, 64);
    }
  }
  if (lane == 0) {
#pragma unroll
    for (int p = 0; p < LG_PTS; ++p) {
      sh[wv][p] = s1[p];
      sh[wv][LG_PTS + p] = s2[p];
    }
  }
  __syncthreads();
  if (threadIdx.x < 2 * LG_PTS) {
    double t = 0.0;
    for (int q = 0; q < LP_BS / 64; ++q) t += sh[q][threadIdx.x];
    part[(long)threadIdx.x * gridDim.x + blockIdx.x] = t;
  }
}

// The two sums at each point (8 threads per sum, strided, then combined in
// a fixed order), the angle test and the new bracket.
__global__ __launch_bounds__(LP_BS) void k_lg_pick(int nblk, const double* __restrict__ part,
                                                   double cmax, LgState* st) {
  __shared__ double tot[2 * LG_PTS];
  const int t = threadIdx.x, q = t >> 3, r = t & 7;
  const unsigned long long lo = st->lo, hi = st->hi;
  if (hi - lo <= 1ull) return;  // converged (uniform)
  double s = 0.0;
  if (q < 2 * LG_PTS)
    for (int j = r; j < nblk; j += 8 * 16) {
      double v[16];
#pragma unroll
      for (int u = 0; u < 16; ++u) v[u] = j + 8 * u < nblk ? part[(long)q * nblk + j + 8 * u] : 0.0;
#pragma unroll
      for (int u = 0; u < 16; ++u) s += v[u];
    }
#pragma unroll
  for (int off = 4; off > 0; off >>= 1) s += __shfl_down(s, off, 8);
  if (q < 2 * LG_PTS && r == 0) tot[q] = s;
  __syncthreads();
  if (t == 0) {
    const double gn = sqrt(st->wsum);
    unsigned long long nlo = lo, nhi = hi;
    for (int p = 0; p < LG_PTS; ++p) {
      const double xp = lg_point(lo, hi, p + 1);
      const unsigned long long xb = (unsigned long long)__double_as_longlong(xp);
      if (xb <= nlo || xb >= nhi) continue;
      // the items outside the bracket once compacted (zeros before)
      const double s1 = tot[p] + (st->c1 + xp * st->whi);
      const double s2 = tot[LG_PTS + p] + (st->c2 + xp * xp * st->whi);
      const double c = s1 / (gn * sqrt(s2));
      if (c > cmax)
        nlo = xb;
      else
        nhi = xb;
    }
    st->lo = nlo;
    st->hi = nhi;
  }
}

// Compaction of the search once the bracket (lo, hi) is narrow: items below
// it enter every later sum as constants (g^2 alpha, g^2 alpha^2), items above
// it as g^2 x and g^2 x^2; only the items inside are kept, in index order.
__device__ __forceinline__ int lg_side(double a, unsigned long long lo, unsigned long long hi) {
  const unsigned long long b = (unsigned long long)__double_as_longlong(a);
  return b <= lo ? -1 : (b >= hi ? 1 : 0);
}
__global__ __launch_bounds__(LP_BS) void k_lg_cls(long n, const double* __restrict__ alpha,
                                                  const double* __restrict__ w, const LgState* st,
                                                  double* __restrict__ part,
                                                  double* __restrict__ counts) {
  __shared__ double sh[LP_BS / 64];
  const unsigned long long lo = st->lo, hi = st->hi;
  double cnt = 0.0, c1 = 0.0, c2 = 0.0, wh = 0.0;
  const long stride = (long)gridDim.x * LP_BS;
  for (long i = (long)blockIdx.x * LP_BS + threadIdx.x; i < n; i += stride) {
    const double a = alpha[i], wi = w[i];
    const int sd = lg_side(a, lo, hi);
    if (sd < 0) {
      c1 += wi * a;
      c2 += wi * a * a;
    } else if (sd > 0) {
      wh += wi;
    } else {
      cnt += 1.0;
    }
  }
  cnt = block_sum_lp(cnt, sh);
  c1 = block_sum_lp(c1, sh);
  c2 = block_sum_lp(c2, sh);
  wh = block_sum_lp(wh, sh);
  if (threadIdx.x == 0) {
    counts[blockIdx.x] = cnt;
    part[gridDim.x + blockIdx.x] = c1;
    part[2 * gridDim.x + blockIdx.x] = c2;
    part[3 * gridDim.x + blockIdx.x] = wh;
  }
}
// The constants and the number of items inside the bracket, in block order
// (the per-block counts are then scanned in place by k_lp_tiescan).
__global__ __launch_bounds__(LP_BS) void k_lg_cls_fin(int nblk, const double* __restrict__ part,
                                                      const double* __restrict__ counts,
                                                      LgState* st) {
  __shared__ double sh[LP_BS / 64];
  double v[4] = {0.0, 0.0, 0.0, 0.0};
  for (int j = threadIdx.x; j < nblk; j += LP_BS) {
    v[0] += counts[j];
    for (int q = 1; q < 4; ++q) v[q] += part[q * nblk + j];
  }
  const double m = block_sum_lp(v[0], sh);
  const double c1 = block_sum_lp(v[1], sh);
  const double c2 = block_sum_lp(v[2], sh);
  const double wh = block_sum_lp(v[3], sh);
  if (threadIdx.x == 0) {
    st->c1 = c1;
    st->c2 = c2;
    st->whi = wh;
    st->mid = m;
  }
}
// The items inside the bracket as (alpha, g^2) pairs, in the order of the
// grid-stride walk of k_lg_cls (block by block, then iteration, then thread).
__global__ __launch_bounds__(LP_BS) void k_lg_cmp_write(long n, const double* __restrict__ alpha,
                                                        const double* __restrict__ w,
                                                        const LgState* st,
                                                        const double* __restrict__ off,
                                                        double* __restrict__ pairs) {
  __shared__ int wc[LP_BS / 64];
  const unsigned long long lo = st->lo, hi = st->hi;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  long pos = (long)off[blockIdx.x];
  const long stride = (long)gridDim.x * LP_BS;
  for (long base = (long)blockIdx.x * LP_BS; base < n; base += stride) {
    const long i = base + threadIdx.x;
    double a = 0.0, wi = 0.0;
    bool in = false;
    if (i < n) {
      a = alpha[i];
      wi = w[i];
      in = lg_side(a, lo, hi) == 0;
    }
    const unsigned long long m = __ballot(in);
    const int below = __popcll(m & ((1ull << lane) - 1ull));
    if (lane == 0) wc[wv] = __popcll(m);
    __syncthreads();
    long before = 0, total = 0;
    for (int q = 0; q < LP_BS / 64; ++q) {
      if (q < wv) before += wc[q];
      total += wc[q];
    }
    if (in) {
      const long j = pos + before + below;
      pairs[2 * j] = a;
      pairs[2 * j + 1] = wi;
    }
    pos += total;
    __syncthreads();
  }
}

__global__ void k_lg_uncompact(LgState* st) {
  if (threadIdx.x == 0) {
    st->c1 = 0.0;
    st->c2 = 0.0;
    st->whi = 0.0;
  }
}

// alpha~ = the largest alpha_i in (0, lo]: block partial maxima, then one block.
__global__ __launch_bounds__(LP_BS) void k_lg_best(long n, const double* __restrict__ alpha,
                                                   const LgState* st, double* __restrict__ part) {
  __shared__ double sh[LP_BS / 64];
  const double lim = __longlong_as_double((long long)st->lo);
  double b = 0.0;
  const long stride = (long)gridDim.x * LP_BS;
  for (long i = (long)blockIdx.x * LP_BS + threadIdx.x; i < n; i += stride) {
    const double a = alpha[i];
    if (a > 0.0 && a <= lim) b = fmax(b, a);
  }
  b = block_max_lp(b, sh);
  if (threadIdx.x == 0) part[blockIdx.x] = b;
}
__global__ __launch_bounds__(LP_BS) void k_lg_best_fin(int nblk, const double* __restrict__ part,
                                                       LgState* st) {
  __shared__ double sh[LP_BS / 64];
  double b = 0.0;
  for (int j = threadIdx.x; j < nblk; j += LP_BS) b = fmax(b, part[j]);
  b = block_max_lp(b, sh);
  if (threadIdx.x == 0) st->alpha = b;
}

// rho~: the bound for alpha_i <= alpha~, rho - alpha~ g (multiply, then
// subtract) for the rest, clipped to [0, 1].
__global__ __launch_bounds__(LP_BS) void k_lg_apply(long n, const double* __restrict__ rho,
                                                    const double* __restrict__ g,
                                                    const double* __restrict__ alpha,
                                                    const LgState* st, double* __restrict__ out) {
#pragma clang fp contract(off)
  const long i = (long)blockIdx.x * LP_BS + threadIdx.x;
  if (i >= n) return;
  const double at = st->alpha;
  const double r = rho[i], gi = g[i];
  double v;
  if (at == 0.0) {
    v = r;
  } else if (gi != 0.0 && alpha[i] <= at) {
    v = gi > 0.0 ? 0.0 : 1.0;
  } else {
    const double step = at * gi;
    v = r - step;
  }
  out[i] = fmin(fmax(v, 0.0), 1.0);
}
}  // namespace

Lp::Lp(long n, int device) : n_(n), device_(device) {
  if (n < 1 || n > (1L << 31)) throw Error(MGCG_EINVAL, "LP size must lie in 1..2^31");
  nb_ = (int)((n + LP_BS - 1) / LP_BS);
  hist_shape(nb_, &ch_, &nh_);
  nr_ = (nh_ + LP_ROWS - 1) / LP_ROWS;
  ns_ = nb_ < LP_SUM_BLOCKS ? nb_ : LP_SUM_BLOCKS;
  MGCG_HIP(hipSetDevice(device_));
  bytes_ = device_bytes(n);
  if (hipMalloc(&arena_, bytes_) != hipSuccess) {
    (void)hipGetLastError();
    arena_ = nullptr;
    throw Error(MGCG_ENOMEM, "LP scratch allocation failed");
  }
  char* p = (char*)arena_;
  auto take = [&](size_t b) {
    char* q = p;
    p += (b + 255) / 256 * 256;
    return (void*)q;
  };
  key_ = (unsigned long long*)take((size_t)n * 8);
  cap_ = (double*)take((size_t)n * 8);
  part_ = (double*)take((size_t)nb_ * 3 * 8);
  bins_ = (double*)take((size_t)nh_ * 256 * 8);
  red_ = (double*)take((size_t)nr_ * 256 * 8);
  tsum_ = (double*)take((size_t)nb_ * 8);
  info_ = (double*)take(4 * 8);
  st_ = take(sizeof(LpState));
  if (hipHostMalloc((void**)&hst_, 256, hipHostMallocDefault) != hipSuccess) {
    (void)hipGetLastError();
    (void)hipFree(arena_);
    arena_ = nullptr;
    throw Error(MGCG_ENOMEM, "LP host buffer allocation failed");
  }
}

// Chunks of LP_BS items per block of the digit passes: enough blocks to fill
// the chip (about 1024), at most 8 chunks each.
void Lp::hist_shape(int nb, int* ch, int* nh) {
  int c = nb / 1024;
  c = c < 1 ? 1 : (c > LP_CH ? LP_CH : c);
  *ch = c;
  *nh = (nb + c - 1) / c;
}

size_t Lp::device_bytes(long n) {
  const long nb = (n + LP_BS - 1) / LP_BS;
  int ch, nh;
  hist_shape((int)nb, &ch, &nh);
  const long nr = (nh + LP_ROWS - 1) / LP_ROWS;
  auto r = [](size_t b) { return (b + 255) / 256 * 256; };
  return r((size_t)n * 8) * 2 + r((size_t)nb * 24) + r((size_t)nh * 2048) + r((size_t)nr * 2048) +
         r((size_t)nb * 8) + r(32) + r(sizeof(LpState));
}

Lp::~Lp() {
  (void)hipSetDevice(device_);
  (void)hipStreamSynchronize(stream_);
  if (arena_) (void)hipFree(arena_);
  if (hst_) (void)hipHostFree(hst_);
}

void Lp::set_stream(hipStream_t s) {
  MGCG_HIP(hipSetDevice(device_));
  MGCG_HIP(hipStreamSynchronize(stream_));
  stream_ = s;
}

void Lp::solve(const double* g, const double* a, const double* x, const unsigned char* fixed,
               double b, double delta, double xl, double xu, double* s, mgcg_lp_info* info,
               int mem) {
  if (!g || !a || !x || !s) throw Error(MGCG_EINVAL, "null vector");
  if (mem != MGCG_MEM_HOST && mem != MGCG_MEM_DEVICE) throw Error(MGCG_EINVAL, "bad mem flag");
  if (!(delta > 0.0) || !std::isfinite(delta) || !std::isfinite(b) || !std::isfinite(xl) ||
      !std::isfinite(xu) || !(xl <= xu))
    throw Error(MGCG_EINVAL, "bad LP scalars (delta > 0, finite b, x_l <= x_u)");
  MGCG_HIP(hipSetDevice(device_));
  const double *dg = g, *da = a, *dx = x;
  double* ds = s;
  void* stage = nullptr;
  struct Free {
    void*& p;
    ~Free() {
      if (p) (void)hipFree(p);
    }
  } fr{stage};
  if (mem == MGCG_MEM_HOST) {
    if (hipMalloc(&stage, (size_t)n_ * 8 * 4 + (fixed ? (size_t)n_ : 0)) != hipSuccess) {
      (void)hipGetLastError();
      stage = nullptr;
      throw Error(MGCG_ENOMEM, "LP staging allocation failed");
    }
    double* base = (double*)stage;
    MGCG_HIP(hipMemcpyAsync(base, g, (size_t)n_ * 8, hipMemcpyHostToDevice, stream_));
    MGCG_HIP(hipMemcpyAsync(base + n_, a, (size_t)n_ * 8, hipMemcpyHostToDevice, stream_));
    MGCG_HIP(hipMemcpyAsync(base + 2 * n_, x, (size_t)n_ * 8, hipMemcpyHostToDevice, stream_));
    dg = base;
    da = base + n_;
    dx = base + 2 * n_;
    ds = base + 3 * n_;
    if (fixed) {
      unsigned char* df = (unsigned char*)(base + 4 * n_);
      MGCG_HIP(hipMemcpyAsync(df, fixed, (size_t)n_, hipMemcpyHostToDevice, stream_));
      fixed = df;
    }
  }
  LpState* st = (LpState*)st_;
  MGCG_HIP(hipMemsetAsync(st, 0, sizeof(LpState), stream_));
  hipLaunchKernelGGL(k_lp_prep, dim3(nb_), dim3(LP_BS), 0, stream_, n_, dg, da, dx, delta, xl, xu,
                     fixed, key_, cap_, part_, st);
  hipLaunchKernelGGL(k_lp_budget, dim3(1), dim3(LP_BS), 0, stream_, n_, nb_, b,
                     (const double*)part_, st);
  // both branches are launched; the feasibility flag in the state selects,
  // on the device, which one runs (no host round trip in between)
  for (int d = 0; d < 8; ++d) {
    hipLaunchKernelGGL(k_lp_hist<false>, dim3(nh_), dim3(LP_BS), 0, stream_, n_, d, ch_,
                       (const unsigned long long*)key_, (const double*)cap_, (const LpState*)st,
                       bins_);
    hipLaunchKernelGGL(k_lp_reduce, dim3(nr_), dim3(LP_BS), 0, stream_, nh_,
                       (const double*)bins_, red_, (const LpState*)st);
    hipLaunchKernelGGL(k_lp_pick, dim3(1), dim3(LP_BS), 0, stream_, nr_, d, (const double*)red_,
                       st);
  }
  hipLaunchKernelGGL(k_lp_tiesum<false>, dim3(nb_), dim3(LP_BS), 0, stream_, n_,
                     (const unsigned long long*)key_, (const double*)cap_, (const LpState*)st,
                     tsum_);
  hipLaunchKernelGGL(k_lp_tiescan, dim3(1), dim3(LP_BS), 0, stream_, nb_, tsum_,
                     (const LpState*)st);
  hipLaunchKernelGGL(k_lp_fill, dim3(nb_), dim3(LP_BS), 0, stream_, n_, dg, da, dx, delta, xl, xu,
                     fixed,
                     (const unsigned long long*)key_, (const double*)cap_, (const double*)tsum_,
                     (const LpState*)st, ds, part_);
  hipLaunchKernelGGL(k_lp_box, dim3(nb_), dim3(LP_BS), 0, stream_, n_, dg, da, dx, delta, xl, xu,
                     fixed, (const LpState*)st, ds, part_);
  hipLaunchKernelGGL(k_lp_info, dim3(1), dim3(LP_BS), 0, stream_, nb_, (const double*)part_, info_);
  MGCG_HIP(hipGetLastError());
  if (mem == MGCG_MEM_HOST)
    MGCG_HIP(hipMemcpyAsync(s, ds, (size_t)n_ * 8, hipMemcpyDeviceToHost, stream_));
  MGCG_HIP(hipMemcpyAsync(hst_, info_, 3 * 8, hipMemcpyDeviceToHost, stream_));
  MGCG_HIP(hipMemcpyAsync((char*)hst_ + 64, st, sizeof(LpState), hipMemcpyDeviceToHost, stream_));
  MGCG_HIP(hipStreamSynchronize(stream_));
  LpState e;
  std::memcpy(&e, (char*)hst_ + 64, sizeof e);
  // (on bad input every kernel ran on sanitised values: capacity 0, ratio 0)
  if (e.bad) throw Error(MGCG_EINVAL, "LP input with a non-positive constraint gradient or a non-finite value");
  const bool feasible = e.feasible != 0;
  if (info) {
    double v[3];
    std::memcpy(v, hst_, sizeof v);
    info->gts = v[0];
    info->ats = v[1];
    info->s_inf = v[2];
    info->feasible = feasible ? 1 : 0;
    info->budget = e.budget;
    info->lambda = feasible ? key_ratio_host(e.prefix) : std::nan("");
  }
}

double Lp::key_ratio_host(unsigned long long k) {
  unsigned long long u = ~k;
  u = (u >> 63) ? (u & 0x7FFFFFFFFFFFFFFFull) : ~u;
  double r;
  std::memcpy(&r, &u, 8);
  return r;
}


// ---- thresholding (Sec. 5) on the same scratch

namespace {
struct Staged {
  void* p = nullptr;
  ~Staged() {
    if (p) (void)hipFree(p);
  }
};
}  // namespace

// Device copies of host inputs (count vectors of n) and a device output.
void Lp::stage_io(int mem, int nin, const double* const* in, const double** din, double* out,
                  double** dout, void** stage) {
  if (mem != MGCG_MEM_HOST && mem != MGCG_MEM_DEVICE) throw Error(MGCG_EINVAL, "bad mem flag");
  for (int q = 0; q < nin; ++q)
    if (!in[q]) throw Error(MGCG_EINVAL, "null vector");
  if (mem == MGCG_MEM_DEVICE) {
    for (int q = 0; q < nin; ++q) din[q] = in[q];
    if (dout) *dout = out;
    return;
  }
  if (hipMalloc(stage, (size_t)n_ * 8 * (nin + 1)) != hipSuccess) {
    (void)hipGetLastError();
    *stage = nullptr;
    throw Error(MGCG_ENOMEM, "staging allocation failed");
  }
  double* base = (double*)*stage;
  for (int q = 0; q < nin; ++q) {
    MGCG_HIP(hipMemcpyAsync(base + q * n_, in[q], (size_t)n_ * 8, hipMemcpyHostToDevice, stream_));
    din[q] = base + q * n_;
  }
  if (dout) *dout = base + nin * n_;
}

void Lp::select_top(const double* v, long k, double* out, int mem) {
  if (!out) throw Error(MGCG_EINVAL, "null vector");
  if (k < 0 || k > n_) throw Error(MGCG_EINVAL, "k outside 0..n");
  MGCG_HIP(hipSetDevice(device_));
  Staged sg;
  const double* din[1];
  double* dout = nullptr;
  const double* in[1] = {v};
  stage_io(mem, 1, in, din, out, &dout, &sg.p);
  LpState* st = (LpState*)st_;
  MGCG_HIP(hipMemsetAsync(st, 0, sizeof(LpState), stream_));
  hipLaunchKernelGGL(k_sel_prep, dim3(nb_), dim3(LP_BS), 0, stream_, n_, din[0], key_, st);
  hipLaunchKernelGGL(k_sel_budget, dim3(1), dim3(64), 0, stream_, (double)k, st);
  for (int d = 0; d < 8; ++d) {
    hipLaunchKernelGGL(k_lp_hist<true>, dim3(nh_), dim3(LP_BS), 0, stream_, n_, d, ch_,
                       (const unsigned long long*)key_, (const double*)cap_, (const LpState*)st,
                       bins_);
    hipLaunchKernelGGL(k_lp_reduce, dim3(nr_), dim3(LP_BS), 0, stream_, nh_, (const double*)bins_,
                       red_, (const LpState*)st);
    hipLaunchKernelGGL(k_lp_pick, dim3(1), dim3(LP_BS), 0, stream_, nr_, d, (const double*)red_, st);
  }
  hipLaunchKernelGGL(k_lp_tiesum<true>, dim3(nb_), dim3(LP_BS), 0, stream_, n_,
                     (const unsigned long long*)key_, (const double*)cap_, (const LpState*)st, tsum_);
  hipLaunchKernelGGL(k_lp_tiescan, dim3(1), dim3(LP_BS), 0, stream_, nb_, tsum_,
                     (const LpState*)st);
  hipLaunchKernelGGL(k_sel_fill, dim3(nb_), dim3(LP_BS), 0, stream_, n_,
                     (const unsigned long long*)key_, (const double*)tsum_, (const LpState*)st, dout);
  MGCG_HIP(hipGetLastError());
  MGCG_HIP(hipMemcpyAsync(hst_, st, sizeof(LpState), hipMemcpyDeviceToHost, stream_));
  if (mem == MGCG_MEM_HOST)
    MGCG_HIP(hipMemcpyAsync(out, dout, (size_t)n_ * 8, hipMemcpyDeviceToHost, stream_));
  MGCG_HIP(hipStreamSynchronize(stream_));
  LpState h;
  std::memcpy(&h, hst_, sizeof h);
  if (h.bad) throw Error(MGCG_EINVAL, "non-finite value");
}

void Lp::round_bounds(const double* r, double lo, double hi, double* out, int mem) {
  if (!out) throw Error(MGCG_EINVAL, "null vector");
  MGCG_HIP(hipSetDevice(device_));
  Staged sg;
  const double* din[1];
  double* dout = nullptr;
  const double* in[1] = {r};
  stage_io(mem, 1, in, din, out, &dout, &sg.p);
  hipLaunchKernelGGL(k_round, dim3(nb_), dim3(LP_BS), 0, stream_, n_, din[0], lo, hi, dout);
  MGCG_HIP(hipGetLastError());
  if (mem == MGCG_MEM_HOST)
    MGCG_HIP(hipMemcpyAsync(out, dout, (size_t)n_ * 8, hipMemcpyDeviceToHost, stream_));
  MGCG_HIP(hipStreamSynchronize(stream_));
}

double Lp::angle_cos(const double* gl, const double* d, int mem) {
  MGCG_HIP(hipSetDevice(device_));
  Staged sg;
  const double* din[2];
  const double* in[2] = {gl, d};
  stage_io(mem, 2, in, din, nullptr, nullptr, &sg.p);
  hipLaunchKernelGGL(k_dot3, dim3(ns_), dim3(LP_BS), 0, stream_, n_, din[0], din[1], part_);
  hipLaunchKernelGGL(k_sum3, dim3(1), dim3(LP_BS), 0, stream_, ns_, (const double*)part_, info_);
  MGCG_HIP(hipGetLastError());
  MGCG_HIP(hipMemcpyAsync(hst_, info_, 24, hipMemcpyDeviceToHost, stream_));
  MGCG_HIP(hipStreamSynchronize(stream_));
  double v[3];
  std::memcpy(v, hst_, sizeof v);
  return -v[0] / (std::sqrt(v[1]) * std::sqrt(v[2]));
}

double Lp::heaviside(const double* r, double beta, double* out, int mem, int* iters) {
  if (!out) throw Error(MGCG_EINVAL, "null vector");
  if (!(beta > 0.0) || !std::isfinite(beta)) throw Error(MGCG_EINVAL, "beta must be positive");
  MGCG_HIP(hipSetDevice(device_));
  Staged sg;
  const double* din[1];
  double* dout = nullptr;
  const double* in[1] = {r};
  stage_io(mem, 1, in, din, out, &dout, &sg.p);
  // Newton's method on f(eta) = sum h - sum rho from eta = 1/2 with the
  // bracket of the sign change (f(0) > 0 > f(1)); the midpoint when a step
  // leaves the bracket; stop at |delta eta| <= 1e-14 or |f| <= 1e-13 sum rho
  double lo = 0.0, hi = 1.0, eta = 0.5;
  int it = 0;
  for (; it < 100; ++it) {
    hipLaunchKernelGGL(k_hv_sums, dim3(ns_), dim3(LP_BS), 0, stream_, n_, din[0], beta, eta,
                       part_);
    hipLaunchKernelGGL(k_sum3, dim3(1), dim3(LP_BS), 0, stream_, ns_, (const double*)part_, info_);
    MGCG_HIP(hipGetLastError());
    MGCG_HIP(hipMemcpyAsync(hst_, info_, 24, hipMemcpyDeviceToHost, stream_));
    MGCG_HIP(hipStreamSynchronize(stream_));
    double v[3];
    std::memcpy(v, hst_, sizeof v);
    const double f = v[0] - v[2];
    if (std::fabs(f) <= 1e-13 * v[2]) break;
    if (f > 0.0)
      lo = eta;
    else
      hi = eta;
    double nxt = v[1] != 0.0 ? eta - f / v[1] : 0.5 * (lo + hi);
    if (!(lo < nxt && nxt < hi)) nxt = 0.5 * (lo + hi);
    const bool done = std::fabs(nxt - eta) <= 1e-14;
    eta = nxt;
    if (done) break;
  }
  hipLaunchKernelGGL(k_hv_apply, dim3(ns_), dim3(LP_BS), 0, stream_, n_, din[0], beta, eta, dout);
  MGCG_HIP(hipGetLastError());
  if (mem == MGCG_MEM_HOST)
    MGCG_HIP(hipMemcpyAsync(out, dout, (size_t)n_ * 8, hipMemcpyDeviceToHost, stream_));
  MGCG_HIP(hipStreamSynchronize(stream_));
  if (iters) *iters = it;
  return eta;
}


double Lp::lagrangian(const double* rho, const double* gl, double vu, double vl, double cmax,
                      double* out, int mem) {
  if (!out) throw Error(MGCG_EINVAL, "null vector");
  if (!std::isfinite(vu) || !std::isfinite(vl) || !std::isfinite(cmax))
    throw Error(MGCG_EINVAL, "non-finite safeguard or angle");
  MGCG_HIP(hipSetDevice(device_));
  Staged sg;
  const double* din[2];
  double* dout = nullptr;
  const double* in[2] = {rho, gl};
  stage_io(mem, 2, in, din, out, &dout, &sg.p);
  LpState* st = (LpState*)st_;
  LgState* lg = (LgState*)st_;
  double* alpha = (double*)key_;
  MGCG_HIP(hipMemsetAsync(st, 0, sizeof(LpState), stream_));
  hipLaunchKernelGGL(k_lg_prep, dim3(ns_), dim3(LP_BS), 0, stream_, n_, din[0], din[1], vu, vl,
                     alpha, cap_, part_, st);
  MGCG_HIP(hipGetLastError());
  MGCG_HIP(hipMemcpyAsync(hst_, st, sizeof(LpState), hipMemcpyDeviceToHost, stream_));
  MGCG_HIP(hipStreamSynchronize(stream_));
  LpState h;
  std::memcpy(&h, hst_, sizeof h);
  if (h.bad) throw Error(MGCG_EINVAL, "non-finite density or gradient");
  hipLaunchKernelGGL(k_lg_init, dim3(1), dim3(LP_BS), 0, stream_, ns_, (const double*)part_, lg);
  // bins_ holds the split partials (2 LG_PTS per block) in front and, after
  // LG_FULL passes over every item, the items still inside the bracket
  double* pairs = bins_ + (size_t)2 * LG_PTS * ns_;
  const long cap_pairs = ((long)nh_ * 256 - 2L * LG_PTS * ns_) / 2;
  int pass = 0;
  for (; pass < LG_FULL; ++pass) {
    hipLaunchKernelGGL(k_lg_split, dim3(ns_), dim3(LP_BS), 0, stream_, n_, (const double*)alpha,
                       (const double*)cap_, 1, (const LgState*)lg, bins_);
    hipLaunchKernelGGL(k_lg_pick, dim3(1), dim3(LP_BS), 0, stream_, ns_, (const double*)bins_,
                       cmax, lg);
  }
  hipLaunchKernelGGL(k_lg_cls, dim3(ns_), dim3(LP_BS), 0, stream_, n_, (const double*)alpha,
                     (const double*)cap_, (const LgState*)lg, bins_, part_);
  hipLaunchKernelGGL(k_lg_cls_fin, dim3(1), dim3(LP_BS), 0, stream_, ns_, (const double*)bins_,
                     (const double*)part_, lg);
  hipLaunchKernelGGL(k_lp_tiescan, dim3(1), dim3(LP_BS), 0, stream_, ns_, part_,
                     (const LpState*)nullptr);
  MGCG_HIP(hipGetLastError());
  MGCG_HIP(hipMemcpyAsync(hst_, lg, sizeof(LgState), hipMemcpyDeviceToHost, stream_));
  MGCG_HIP(hipStreamSynchronize(stream_));
  LgState mid;
  std::memcpy(&mid, hst_, sizeof mid);
  const long m = (long)mid.mid;
  if (m <= cap_pairs) {
    hipLaunchKernelGGL(k_lg_cmp_write, dim3(ns_), dim3(LP_BS), 0, stream_, n_,
                       (const double*)alpha, (const double*)cap_, (const LgState*)lg,
                       (const double*)part_, pairs);
    long nsc = (m + LP_BS * 4 - 1) / (LP_BS * 4);
    nsc = nsc < 1 ? 1 : (nsc > ns_ ? ns_ : nsc);
    for (; pass < 16; ++pass) {
      hipLaunchKernelGGL(k_lg_split, dim3(nsc), dim3(LP_BS), 0, stream_, m,
                         (const double*)pairs, (const double*)pairs + 1, 2, (const LgState*)lg,
                         bins_);
      hipLaunchKernelGGL(k_lg_pick, dim3(1), dim3(LP_BS), 0, stream_, (int)nsc,
                         (const double*)bins_, cmax, lg);
    }
  } else {
    // too many items left inside the bracket for the scratch: no compaction
    hipLaunchKernelGGL(k_lg_uncompact, dim3(1), dim3(64), 0, stream_, lg);
    for (; pass < 16; ++pass) {
      hipLaunchKernelGGL(k_lg_split, dim3(ns_), dim3(LP_BS), 0, stream_, n_, (const double*)alpha,
                         (const double*)cap_, 1, (const LgState*)lg, bins_);
      hipLaunchKernelGGL(k_lg_pick, dim3(1), dim3(LP_BS), 0, stream_, ns_, (const double*)bins_,
                         cmax, lg);
    }
  }
  hipLaunchKernelGGL(k_lg_best, dim3(ns_), dim3(LP_BS), 0, stream_, n_, (const double*)alpha,
                     (const LgState*)lg, part_);
  hipLaunchKernelGGL(k_lg_best_fin, dim3(1), dim3(LP_BS), 0, stream_, ns_, (const double*)part_,
                     lg);
  hipLaunchKernelGGL(k_lg_apply, dim3(nb_), dim3(LP_BS), 0, stream_, n_, din[0], din[1],
                     (const double*)alpha, (const LgState*)lg, dout);
  MGCG_HIP(hipGetLastError());
  if (mem == MGCG_MEM_HOST)
    MGCG_HIP(hipMemcpyAsync(out, dout, (size_t)n_ * 8, hipMemcpyDeviceToHost, stream_));
  MGCG_HIP(hipMemcpyAsync(hst_, lg, sizeof(LgState), hipMemcpyDeviceToHost, stream_));
  MGCG_HIP(hipStreamSynchronize(stream_));
  LgState r;
  std::memcpy(&r, hst_, sizeof r);
  return r.alpha;
}

// ---- step control of Algorithm 2 (host)

int slp_decide(mgcg_slp_ctrl* c, double f0, double f1, double c0, double c1, double gts, double ats,
               double s_inf, double* theta, double* a_red, double* p_red) {
  // predicted reductions of the linear model: M(x, s) = (a^T s + c)^2 / 2
  const double m0 = 0.5 * c0 * c0, m1 = 0.5 * (ats + c0) * (ats + c0);
  // P_opt is the predicted reduction of f, -g^T s (P_red = theta P_opt +
  // (1 - theta) P_fsb)
  const double p_fsb = m0 - m1, p_opt = -gts;
  // eqs. (theta1), (theta2)
  const double large = (1.0 + c->N / std::pow((double)c->k + 1.0, 1.1)) * c->theta_min_hist;
  const double sup = p_opt <= 0.5 * p_fsb ? 0.5 * p_fsb / (p_fsb - p_opt) : 1.0;
  const double th = std::fmin(std::fmin(large, sup), c->theta_max);
  const double ar = th * (f0 - f1) + (1.0 - th) * (0.5 * c0 * c0 - 0.5 * c1 * c1);
  const double pr = -th * gts + (1.0 - th) * p_fsb;
  if (theta) *theta = th;
  if (a_red) *a_red = ar;
  if (p_red) *p_red = pr;
  if (ar < 0.1 * pr) {  // reject: shrink the trust region
    c->delta = std::fmin(0.25 * s_inf, 0.1 * c->delta);
    c->theta_max = th;
    return 0;
  }
  if (ar >= 0.5 * pr) c->delta = std::fmin(2.0 * c->delta, c->box_inf);
  c->delta = std::fmax(c->delta, c->delta_min);
  c->theta_min_hist = std::fmin(c->theta_min_hist, th);
  c->theta_max = 1.0;
  c->k += 1;
  return 1;
}

}  // namespace mgcg
