// RANSAC hypothesise-and-verify on the GPU.
//
// Work item = (pair, block of HB hypotheses). A workgroup (256 threads; 512
// for the fused single pair) solves its HB hypotheses (one per thread) into
// LDS, then scores them against the pair's points: each lane holds P correspondences in registers, every lane
// reads the hypothesis from LDS, the inlier test runs per (hypothesis, point)
// and counts come from a wavefront ballot + popcount. The argmax is over a
// packed (count, ~index) key.
//
// Forms:
//  * fused single pair: grid = hypothesis blocks, each writing its best key;
//    a second kernel reduces them and writes the mask;
//  * plain single pair: solve all -> H buffer, score, argmax, mask kernels;
//  * batched persistent: CUs x blocks_per_cu workgroups drain an atomic queue
//    of items ordered by pair size (largest first); each item atomicMax-es its
//    key into the pair's; a finish kernel (one workgroup per pair) then
//    recomputes each winner and writes the outputs and masks;
//  * adaptive termination: items are rounds of 64 hypotheses; each writes its
//    round key into a write-once slot and may advance an advisory prefix that
//    lets later rounds be skipped; the finish kernel applies the stopping rule
//    to the slots in order.
// Workgroups exchange nothing but atomics whose results the finish kernel
// reads after the launch boundary, so no fences are needed.
#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <tuple>
#include <vector>

#include "common.hpp"
#include "ransac_dev.hpp"

namespace hg {

constexpr int kThreads = 256;
constexpr int kWaves = kThreads / 64;
// Waves per workgroup of the fused single-pair kernel: 8 (512 threads, two
// workgroups and four waves per SIMD at about two workgroups per CU).
constexpr int kFusedWaves = 8;

struct RansacArgs {
  const float *corr;
  int64_t ld;
  const int64_t *off;      // n_pairs + 1 offsets, or nullptr for one pair of n_single points
  int32_t n_single;
  int32_t n_pairs;
  int32_t n_hyp;
  int32_t n_hb;            // hypothesis blocks per pair
  int64_t n_items;         // n_pairs * n_hb
  float tau;
  float inv_tau;           // 1/tau rounded to float (the scoring form's scale)
  uint32_t k0, k1;         // Philox key (seed low / high word)
  float *best_H;
  int32_t *best_count;
  int32_t *best_hyp;
  uint8_t *mask;
  int32_t *hyp_counts;     // may be null
  unsigned long long *keys;
  uint32_t *queue;
  const int32_t *order;    // pair processing order (largest first), or nullptr
  float *hbuf;             // single pair: every hypothesis's H (9 floats), or nullptr
  unsigned long long *blockbest;   // single pair: best key of each work item, or nullptr
  // adaptive termination (nullptr pst = off): work items are rounds of HB
  // hypotheses; per pair and round the round's best key (write-once slot);
  // per pair the advisory prefix and stopping hint
  struct PairState *pst;
  unsigned long long *rkey;
  int32_t *iorder;         // adaptive: queue position -> pair * n_hb + round, or NULL
  int32_t *n_eval;
  double one_minus_conf;
};

// Advisory state of one pair under adaptive termination, read and written
// only with relaxed atomics. `prefix` = (front << 32) | best count over rounds
// [0, front), extended in order from published round keys (monotone in both
// halves, so atomicMax keeps the furthest one); `stop` = a number of rounds
// after which no round is needed (an exact stopping point or a bound on it;
// atomicMin). Rounds at or past `stop` are skipped or abandoned. Nothing here
// decides a result: the finish kernel re-applies the rule to the published
// round keys in order.
struct PairState {
  unsigned long long prefix;
  uint32_t stop, pad;
};

// Round key slot not yet published (no real key has all bits set).
constexpr unsigned long long kUnpublished = ~0ull;

// Hypotheses per round under adaptive termination (one work item).
constexpr int kRoundHyps = 64;

__device__ __forceinline__ void pair_range(const RansacArgs &a, int p, int64_t &base, uint32_t &n) {
  if (a.off) {
    // clamped into the planes, so that offsets outside them cannot move an access out
    base = min(max(a.off[p], int64_t(0)), a.ld);
    const int64_t e = min(max(a.off[p + 1], base), a.ld);
    const int64_t m = e - base;
    n = m > 0x7FFFFFFF ? 0x7FFFFFFFu : static_cast<uint32_t>(m);
  } else {
    base = 0;
    n = static_cast<uint32_t>(a.n_single);
  }
}

// Maximum of a 64-bit value over the 64 lanes of a wave (result in every lane).
__device__ __forceinline__ unsigned long long wave_max_u64(unsigned long long v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    const unsigned long long w = __shfl_xor(v, o);
    v = w > v ? w : v;
  }
  return v;
}

// Maximum of a float over the 64 lanes of a wave (result in every lane).
__device__ __forceinline__ float wave_max_f32(float v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = fmaxf(v, __shfl_xor(v, o));
  return v;
}

// Rows of points per group in the scoring loop: the unit whose float32
// count is replaced by a float64 recount when a sign in it is not proven.
constexpr int kGroup = 4;

// Groups to recount, listed in LDS by the scoring loop (which leaves their
// points out of its counts) and counted after it, when the loop's point
// registers are free. Entry: the chunk's first point and (hypothesis |
// group << 6 | wave << 9 | rows << 12). n counts every append; past kFixCap
// the list has overflowed and every hypothesis is recounted in float64.
constexpr uint32_t kFixCap = 512;
static_assert(kWaves <= 8 && kFusedWaves <= 8, "a recount entry holds the wave index in 3 bits");
struct FixList {
  uint32_t n;
  uint32_t e[kFixCap][2];
};

// Inliers of H (the float H, given as doubles) among `rows` (<= kGroup) rows
// of 64 points, NW * 64 points apart from point ib of this lane (points
// at or past n excluded), by the float64 test on the operands read from
// memory (every row's loads issued before the first test; 32-bit byte
// offsets from the plane bases, which the pair range keeps below 2^33).
template <int NW>
__device__ __forceinline__ uint32_t count_f64(const RansacArgs &a, const float *X1,
                                              const float *Y1, const float *X2, const float *Y2,
                                              uint32_t ib, uint32_t n, uint32_t rows,
                                              const double *g) {
  float x1[kGroup], y1[kGroup], x2[kGroup], y2[kGroup];
#pragma unroll
  for (int q = 0; q < kGroup; ++q) {
    const uint32_t j = min(ib + q * NW * 64u, n - 1u);   // loads stay inside the pair
    x1[q] = X1[j];
    y1[q] = Y1[j];
    x2[q] = X2[j];
    y2[q] = Y2[j];
  }
  uint32_t c = 0u;
#pragma unroll
  for (int q = 0; q < kGroup; ++q) {
    const uint32_t i = ib + q * NW * 64u;
    const bool in = inlier_f64(g, x1[q], y1[q], x2[q], y2[q], a.tau);
    c += __popcll(__ballot(in && i < n && static_cast<uint32_t>(q) < rows));
  }
  return c;
}

// List length up to which fix_counts recounts every listed group without
// bounding which hypotheses can still reach the best.
constexpr uint32_t kBoundMin = 32;

// After the scoring loop (and a workgroup barrier): apply the listed float64
// recounts to cnt, or on overflow recount every valid hypothesis over all
// points. With `all` false (per-hypothesis counts are not an output), a
// hypothesis is recounted only if it could still reach the best count among
// the hypotheses counted exactly here: its listed points added to its count
// reach that best (ties included). The others keep a count below their true
// one, which stays below the best, so the maximum, its lowest index and the
// mask do not change. The bound costs two barriers and LDS atomics, so with
// at most kBoundMin entries every listed group is recounted instead. ub: LDS
// scratch of HB words. NW: waves per workgroup. Ends with a workgroup barrier.
template <int NW>
__device__ void fix_counts(const RansacArgs &a, int64_t base, uint32_t n, const double (*H0s)[9],
                           FixList *fx, uint64_t vmask, int nh, uint32_t *cnt, bool all,
                           uint32_t *ub) {
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const float *X1 = a.corr + base, *Y1 = a.corr + a.ld + base;
  const float *X2 = a.corr + 2 * a.ld + base, *Y2 = a.corr + 3 * a.ld + base;
  const uint32_t ne = fx->n;
  if (ne <= kFixCap) {
    uint32_t best = 0u;
    const bool bound = !all && ne > kBoundMin;
    if (bound) {
      // ub[h]: the count so far plus the listed points of h
      for (int h = threadIdx.x; h < nh; h += NW * 64) ub[h] = cnt[h];
      __syncthreads();
      for (uint32_t k = threadIdx.x; k < ne; k += NW * 64) {
        const uint32_t w = fx->e[k][1];
        atomicAdd(&ub[w & 63u], ((w >> 12) & 31u) * 64u);
      }
      __syncthreads();
      // the best exact count: valid hypotheses with nothing listed
      const bool exact = lane < nh && ((vmask >> lane) & 1ull) && ub[lane] == cnt[lane];
      uint32_t v = exact ? cnt[lane] : 0u;
#pragma unroll
      for (int o = 32; o > 0; o >>= 1) v = max(v, static_cast<uint32_t>(__shfl_xor(v, o)));
      best = v;
    }
    for (uint32_t k = wave; k < ne; k += NW) {
      const uint32_t c0 = fx->e[k][0], w = fx->e[k][1];
      const uint32_t h = w & 63u, g = (w >> 6) & 7u, wv = (w >> 9) & 7u, rows = (w >> 12) & 31u;
      if (bound && ub[h] < best) continue;   // cannot reach the best
      const uint32_t ib = c0 + (g * kGroup * NW + wv) * 64u + lane;
      const uint32_t c64 = count_f64<NW>(a, X1, Y1, X2, Y2, ib, n, rows, H0s[h]);
      if (lane == 0 && c64) atomicAdd(&cnt[h], c64);
    }
  } else {
    for (int h = wave; h < nh; h += NW) {
      if (!((vmask >> h) & 1ull)) continue;
      uint32_t c = 0u;
      for (uint32_t c0 = 0; c0 < n; c0 += NW * 64u * kGroup)
        for (int wv = 0; wv < NW; ++wv)
          c += count_f64<NW>(a, X1, Y1, X2, Y2, c0 + wv * 64u + lane, n, kGroup, H0s[h]);
      if (lane == 0) cnt[h] = c;
    }
  }
  __syncthreads();
}

// Count, for each hypothesis h < nh whose bit is set in vmask, the inliers
// among the points [base, base + n) held in registers (P per lane); each wave
// adds its counts into cnt[h] (LDS atomics). Hs holds the hypotheses' scoring
// forms. TAIL: the chunk runs past n and lanes beyond it are masked out of the
// ballots.
// Each wave decides its P x 64 points in float32, in groups of kGroup rows,
// and keeps per lane and group the minimum over its points of
// |e32| - |w| k1; where that reaches k0 for some lane (a point whose float32
// sign is not proven, see error_bound), the group is listed in fx for a
// float64 recount after the loop (fix_counts). The error bound's magnitudes
// are the wave's maxima over its points, and its coefficients are computed
// once per chunk, lane h for hypothesis h.
// Under adaptive termination `stop` points at the pair's stopping hint and
// `hb` is this item's round: every 8 hypotheses the wave compares hb with the
// value it loaded at the previous check (the load's latency overlaps the 8
// hypotheses) and gives up a round that is no longer needed (returns false).
// Rounds at or past the hint are never needed, so an abandoned round changes
// no result.
template <int P, bool TAIL, int NW>
__device__ __forceinline__ bool score_chunk(const RansacArgs &a, const float *X1, const float *Y1,
                                            const float *X2, const float *Y2, uint32_t c0,
                                            uint32_t n, const float (*Hs)[9],
                                            uint64_t vmask, int nh, uint32_t *cnt,
                                            FixList *fx, const uint32_t *stop, uint32_t hb) {
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  float x1[P], y1[P], x2[P], y2[P];
  uint64_t live[TAIL ? P : 1];
  float m1 = 0.0f, m2 = 0.0f, m3 = 0.0f, m4 = 0.0f;
#pragma unroll
  for (int p = 0; p < P; ++p) {
    const uint32_t i = c0 + (p * NW + wave) * 64 + lane;
    const uint32_t j = (TAIL && i >= n) ? n - 1u : i;   // every load stays inside the pair
    x1[p] = X1[j];
    y1[p] = Y1[j];
    x2[p] = X2[j] * a.inv_tau;
    y2[p] = Y2[j] * a.inv_tau;
    if (TAIL) live[p] = __ballot(i < n);
    m1 = fmaxf(m1, fabsf(x1[p]));
    m2 = fmaxf(m2, fabsf(y1[p]));
    m3 = fmaxf(m3, fabsf(x2[p]));
    m4 = fmaxf(m4, fabsf(y2[p]));
  }
  m1 = wave_max_f32(m1);
  m2 = wave_max_f32(m2);
  m3 = wave_max_f32(m3);
  m4 = wave_max_f32(m4);
  // lane h: error-bound coefficients of hypothesis h over this wave's points
  float k1v = 0.0f, k0v = 0.0f;
  if (lane < nh) error_bound(Hs[lane], m1, m2, m3, m4, k1v, k0v);
  uint32_t stop_seen =
      stop ? __hip_atomic_load(stop, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) : 0u;
  for (int h = 0; h < nh; ++h) {
    if (stop && (h & 7) == 7) {
      if (hb >= stop_seen) return false;
      stop_seen = __hip_atomic_load(stop, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    if (!((vmask >> h) & 1ull)) continue;
    // H read from LDS by every lane (one address: a broadcast) and used from
    // vector registers; scalar copies would cost a readfirstlane per entry and
    // moves wherever an FMA needs two of them
    float hh[9];
#pragma unroll
    for (int k = 0; k < 9; ++k) hh[k] = Hs[h][k];
    const float k1 = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(k1v), h));
    const float k0 = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(k0v), h));
    // rows in groups of kGroup: per group the float32 count and the minimum
    // over its points of |e32| - |w| k1 (the margin by which the sign is
    // proven); a group with a sign not proven is listed for a float64 recount
    // (which then supplies its whole count) instead of counted here
    uint32_t c = 0;
#pragma unroll
    for (int g = 0; g < (P + kGroup - 1) / kGroup; ++g) {
      uint32_t cg = 0u;
      float slack = __builtin_inff();
#pragma unroll
      for (int q = 0; q < kGroup; ++q) {
        const int p = g * kGroup + q;
        if (p < P) {
          float w;
          const float e = test_f32(hh, x1[p], y1[p], x2[p], y2[p], w);
          uint64_t m = __ballot(e <= 0.0f);
          if (TAIL) m &= live[p];
          cg += __popcll(m);
          slack = fminf(slack, fmaf(-fabsf(w), k1, fabsf(e)));
        }
      }
      if (__builtin_expect(__ballot(slack <= k0) != 0ull, 0)) {
        if (lane == 0) {
          const uint32_t k = atomicAdd(&fx->n, 1u);
          if (k < kFixCap) {
            const uint32_t rows = min(kGroup, P - g * kGroup);
            fx->e[k][0] = c0;
            fx->e[k][1] = static_cast<uint32_t>(h) | (static_cast<uint32_t>(g) << 6) |
                          (static_cast<uint32_t>(wave) << 9) | (rows << 12);
          }
        }
      } else {
        c += cg;
      }
    }
    if (lane == 0 && c) atomicAdd(&cnt[h], c);
  }
  return true;
}

// Full chunks of P points per lane, then (P = 16) chunks of 8, then one
// masked tail chunk of just enough 64-point rows per wave (1 to 8), so that a
// pair's last chunk leaves fewer than NW x 64 lane slots idle (NW: waves per
// workgroup). Counts are integer sums over the points, so the result does not
// depend on the chunking.
template <int P, int NW = kWaves>
__device__ __forceinline__ void score_hyps(const RansacArgs &a, int64_t base, uint32_t n,
                                           const float (*Hs)[9], uint64_t vmask, int nh,
                                           uint32_t *cnt, FixList *fx,
                                           const uint32_t *stop = nullptr,
                                           uint32_t hb = 0u) {
  const float *X1 = a.corr + base, *Y1 = a.corr + a.ld + base;
  const float *X2 = a.corr + 2 * a.ld + base, *Y2 = a.corr + 3 * a.ld + base;
  constexpr uint32_t kChunk = NW * 64 * P;
  constexpr uint32_t kChunk8 = NW * 64 * 8;
  uint32_t c0 = 0;
  for (; c0 + kChunk <= n; c0 += kChunk)
    if (!score_chunk<P, false, NW>(a, X1, Y1, X2, Y2, c0, n, Hs, vmask, nh, cnt, fx, stop, hb))
      return;
  if (P > 8) {
    for (; c0 + kChunk8 <= n; c0 += kChunk8)
      if (!score_chunk<8, false, NW>(a, X1, Y1, X2, Y2, c0, n, Hs, vmask, nh, cnt, fx, stop, hb))
        return;
  }
  if (c0 < n) {
    // fewer than kChunk8 points remain: 1 .. 8 rows of 64 points per wave
    const uint32_t rows = (n - c0 + 63u) / 64u;
    switch ((rows + NW - 1) / NW) {
#define HG_TAIL(R) \
  case R:          \
    score_chunk<R, true, NW>(a, X1, Y1, X2, Y2, c0, n, Hs, vmask, nh, cnt, fx, stop, hb); \
    break;
      HG_TAIL(1)
      HG_TAIL(2)
      HG_TAIL(3)
      HG_TAIL(4)
      HG_TAIL(5)
      HG_TAIL(6)
      HG_TAIL(7)
      default:
        score_chunk<8, true, NW>(a, X1, Y1, X2, Y2, c0, n, Hs, vmask, nh, cnt, fx, stop, hb);
#undef HG_TAIL
    }
  }
}

// Adaptive stopping rule: with eps = best_count / n, enough samples have been
// drawn once (1 - eps^4)^m <= 1 - confidence, i.e. m >= log(1 - confidence) /
// log(1 - eps^4) rounded up (m integer). The power is taken by repeated
// squaring in double.
__device__ __forceinline__ bool enough_samples(uint32_t best_count, uint32_t n, uint32_t m,
                                               double one_minus_conf) {
  if (n == 0u) return false;
  const double eps = static_cast<double>(best_count) / static_cast<double>(n);
  const double e2 = eps * eps;
  const double q = 1.0 - e2 * e2;
  double r = 1.0, b = q;
  for (uint32_t e = m; e; e >>= 1) {
    if (e & 1u) r *= b;
    b *= b;
  }
  return r <= one_minus_conf;
}

#define HG_AGENT __HIP_MEMORY_SCOPE_AGENT

__device__ __forceinline__ uint32_t key_count(unsigned long long k) {
  return k ? static_cast<uint32_t>((k >> 32) - 1ull) : 0u;
}

// Called by one thread after round hb of pair p published `key`. If hb is the
// pair's front, extends the merged prefix over the rounds published since
// (in order), applies the stopping rule at each step, and lowers `stop` to
// the stopping point when it holds, else to the bound that the prefix's best
// count gives (the count only grows and the rule is monotone in it, so the
// rule holds at the latest there). Every value read is final (a slot is
// written once per launch) or the sentinel, so a stale read only means a
// shorter prefix, never a wrong one.
__device__ void adaptive_hint(const RansacArgs &a, int p, uint32_t n_pts, int HB, int hb,
                              unsigned long long key) {
  PairState *st = a.pst + p;
  const unsigned long long w = __hip_atomic_load(&st->prefix, __ATOMIC_RELAXED, HG_AGENT);
  uint32_t f = static_cast<uint32_t>(w >> 32);
  if (f != static_cast<uint32_t>(hb)) return;
  uint32_t bc = static_cast<uint32_t>(w);
  uint32_t s = __hip_atomic_load(&st->stop, __ATOMIC_RELAXED, HG_AGENT);
  const uint32_t n_hyp = static_cast<uint32_t>(a.n_hyp);
  const unsigned long long *rk = a.rkey + static_cast<int64_t>(p) * a.n_hb;
  unsigned long long k = key;
  for (;;) {
    bc = max(bc, key_count(k));
    ++f;
    const uint32_t m = min(f * static_cast<uint32_t>(HB), n_hyp);
    if (m >= n_hyp || enough_samples(bc, n_pts, m, a.one_minus_conf)) {
      s = min(s, f);
      break;
    }
    if (f >= s) break;
    k = __hip_atomic_load(&rk[f], __ATOMIC_RELAXED, HG_AGENT);
    if (k == kUnpublished) break;
  }
  for (uint32_t c = f + 1u; c < s; ++c)
    if (enough_samples(bc, n_pts, min(c * static_cast<uint32_t>(HB), n_hyp), a.one_minus_conf)) {
      s = c;
      break;
    }
  atomicMax(&st->prefix, (static_cast<unsigned long long>(f) << 32) | bc);
  atomicMin(&st->stop, s);
}

// Shared memory of one workgroup.
template <int HB>
struct Smem {
  float H[HB][9];          // scoring form (rows 1-2 scaled by 1/tau)
  double H0[HB][9];        // the float H, as doubles (for the float64 test)
  uint32_t valid[HB];
  uint32_t cnt[HB];
  uint32_t ub[HB];         // scratch of fix_counts
  FixList fix;             // groups to recount in float64
  int64_t item;
  uint32_t skip;
};

// Process one work item: pair rank r, hypothesis block hb (NW waves).
template <int P, int HB, int NW>
__device__ void run_item(const RansacArgs &a, int64_t item, Smem<HB> &sm) {
  // pair-major items (all blocks of the largest pair first), or round-major
  // under adaptive termination (round r of every pair before round r + 1)
  const bool adaptive = a.pst != nullptr;
  int p, hb;
  if (adaptive && a.iorder) {
    // staggered round order (ransac_round_order_kernel); decoded into range
    const uint32_t code = static_cast<uint32_t>(a.iorder[item]);
    p = min(static_cast<int>(code / static_cast<uint32_t>(a.n_hb)), a.n_pairs - 1);
    hb = static_cast<int>(code % static_cast<uint32_t>(a.n_hb));
  } else {
    const int r = static_cast<int>(adaptive ? item % a.n_pairs : item / a.n_hb);
    hb = static_cast<int>(adaptive ? item / a.n_pairs : item % a.n_hb);
    p = a.order ? a.order[r] : r;
  }
  int64_t base;
  uint32_t n;
  pair_range(a, p, base, n);
  if (adaptive) {
    // rounds at or past a known stopping point are not evaluated
    if (threadIdx.x == 0)
      sm.skip = static_cast<uint32_t>(hb) >=
                __hip_atomic_load(&a.pst[p].stop, __ATOMIC_RELAXED, HG_AGENT);
    __syncthreads();
    const bool skip = sm.skip != 0u;
    __syncthreads();
    if (skip) return;
  }
  const int h0 = hb * HB;
  const int nh = min(HB, a.n_hyp - h0);
  // 1. solve this block's hypotheses, one per thread
  if (threadIdx.x < HB) {
    const int t = threadIdx.x;
    uint32_t f = kZeroH;
    if (t < nh) {
      float h[9];
      f = make_hypothesis(a.corr, a.ld, base, n, a.k0, a.k1, static_cast<uint32_t>(h0 + t),
                          static_cast<uint32_t>(p), h);
      score_form(h, a.inv_tau, sm.H[t]);
#pragma unroll
      for (int k = 0; k < 9; ++k) sm.H0[t][k] = h[k];
      if (a.hbuf)
#pragma unroll
        for (int k = 0; k < 9; ++k) a.hbuf[9ll * (h0 + t) + k] = h[k];
    }
    sm.valid[t] = (t < nh && f == 0u) ? 1u : 0u;
    sm.cnt[t] = 0u;
  }
  if (threadIdx.x == 0) sm.fix.n = 0u;
  __syncthreads();
  // 2. score (validity as a wave-uniform bit mask)
  const int lane = threadIdx.x & 63;
  const uint64_t vmask = __ballot(lane < nh && sm.valid[lane] != 0u);
  score_hyps<P, NW>(a, base, n, sm.H, vmask, nh, sm.cnt, &sm.fix,
                adaptive ? &a.pst[p].stop : nullptr, static_cast<uint32_t>(hb));
  __syncthreads();
  fix_counts<NW>(a, base, n, sm.H0, &sm.fix, vmask, nh, sm.cnt, a.hyp_counts != nullptr, sm.ub);
  if (adaptive) {
    // a wave may have given the round up: then it is at or past the stopping
    // round (which only decreases), and nothing of it is published
    if (threadIdx.x == 0)
      sm.skip = static_cast<uint32_t>(hb) >=
                __hip_atomic_load(&a.pst[p].stop, __ATOMIC_RELAXED, HG_AGENT);
    __syncthreads();
    const bool skip = sm.skip != 0u;
    __syncthreads();
    if (skip) return;
  }
  // 3. publish counts and the block's best key (wave 0 holds all HB <= 64)
  if (threadIdx.x < 64) {
    const int t = threadIdx.x;
    unsigned long long key = 0ull;
    if (t < nh) {
      const uint32_t c = sm.cnt[t];
      const bool ok = sm.valid[t] != 0u;
      if (a.hyp_counts)
        a.hyp_counts[static_cast<int64_t>(p) * a.n_hyp + h0 + t] = ok ? static_cast<int32_t>(c) : 0;
      if (ok) key = pack_key(c, static_cast<uint32_t>(h0 + t));
    }
    key = wave_max_u64(key);
    if (t == 0) {
      if (a.blockbest) {
        a.blockbest[item] = key;     // reduced by the mask kernel
      } else if (adaptive) {
        // write-once slot, then the advisory prefix / stopping hint
        __hip_atomic_store(&a.rkey[static_cast<int64_t>(p) * a.n_hb + hb], key, __ATOMIC_RELAXED,
                           HG_AGENT);
        adaptive_hint(a, p, n, HB, hb, key);
      } else if (key != 0ull) {
        atomicMax(&a.keys[p], key);  // the pair's outputs come from the finish kernel
      }
    }
  }
  // Every wave leaves the item here together. Without this barrier the
  // thread-0-only tail above may be folded into the persistent loop so that
  // waves execute the loop's barriers different numbers of times.
  __syncthreads();
}

// Persistent: kThreads threads, at least 5 workgroups per CU. Single pair
// (one work item per workgroup): kFusedWaves waves, at least 2 per CU.
template <int P, int HB, bool PERSISTENT>
__global__ __launch_bounds__(PERSISTENT ? kThreads : kFusedWaves * 64, PERSISTENT ? 5 : 2)
void ransac_kernel(RansacArgs a) {
  __shared__ Smem<HB> sm;
  if (!PERSISTENT) {
    run_item<P, HB, kFusedWaves>(a, blockIdx.x, sm);
    return;
  }
  for (;;) {
    if (threadIdx.x == 0) sm.item = static_cast<int64_t>(atomicAdd(a.queue, 1u));
    __syncthreads();
    const int64_t item = sm.item;
    __syncthreads();
    if (item >= a.n_items) break;
    run_item<P, HB, kWaves>(a, item, sm);
  }
}

// After the persistent kernel (whose keys are then all visible): one workgroup
// per pair writes the pair's best hypothesis, count, index, hypotheses
// evaluated and inlier mask. Fixed count: the pair's key is the atomicMax of
// its blocks' keys. Adaptive termination: the stopping rule applied to the
// published round keys in order, as a sequential loop would (a round before
// the stopping point is always published; if one were missing, n_evaluated
// would read -1).
constexpr int kFinishThreads = 1024;

__global__ __launch_bounds__(kFinishThreads) void ransac_finish_kernel(RansacArgs a) {
  __shared__ float bestH[9];
  __shared__ unsigned long long skey;
  __shared__ int32_t sne;
  const int p = blockIdx.x;
  int64_t base;
  uint32_t n;
  pair_range(a, p, base, n);
  if (a.pst && threadIdx.x < 64) {
    // wave 0: 64 rounds at a time, in order; lane f holds round c0 + f, its
    // prefix maximum (shuffle scan) and whether the rule holds after it
    const int lane = threadIdx.x;
    const uint32_t n_hyp = static_cast<uint32_t>(a.n_hyp);
    const unsigned long long *rk = a.rkey + static_cast<int64_t>(p) * a.n_hb;
    unsigned long long carry = 0ull, key = 0ull;
    int32_t ne = -1;
    for (int c0 = 0; c0 < a.n_hb; c0 += 64) {
      const int f = c0 + lane;
      const unsigned long long k = f < a.n_hb ? rk[f] : kUnpublished;
      const bool pub = k != kUnpublished;
      unsigned long long v = pub ? k : 0ull;
#pragma unroll
      for (int o = 1; o < 64; o <<= 1) {
        const unsigned long long u = __shfl_up(v, o);
        if (lane >= o) v = max(v, u);
      }
      v = max(v, carry);
      const uint32_t m = min(static_cast<uint32_t>(f + 1) * static_cast<uint32_t>(kRoundHyps),
                             n_hyp);
      const bool stop = f < a.n_hb && pub &&
                        (m >= n_hyp || enough_samples(key_count(v), n, m, a.one_minus_conf));
      const uint64_t sb = __ballot(stop), ub = __ballot(f < a.n_hb && !pub);
      if (sb != 0ull) {
        const int fs = __ffsll(static_cast<long long>(sb)) - 1;   // first round where it holds
        // a round before it unpublished cannot happen (reported as -1)
        const bool gap = (ub & ((2ull << fs) - 1ull)) != 0ull;
        const unsigned long long vk = __shfl(v, fs);
        key = vk;
        ne = gap ? -1 : static_cast<int32_t>(min(static_cast<uint32_t>(c0 + fs + 1) *
                                                     static_cast<uint32_t>(kRoundHyps),
                                                 n_hyp));
        break;
      }
      if (ub != 0ull) break;   // unpublished before any stop: -1
      carry = __shfl(v, 63);
    }
    if (lane == 0) {
      skey = key;
      sne = ne;
    }
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    unsigned long long key;
    int32_t ne;
    if (a.pst) {
      key = skey;
      ne = sne;
    } else {
      key = a.keys[p];
      ne = a.n_hyp;
    }
    if (a.n_eval) a.n_eval[p] = ne;
    if (key != 0ull) {
      const uint32_t hyp = 0xFFFFFFFFu - static_cast<uint32_t>(key & 0xFFFFFFFFull);
      // the winner is recomputed (same device function, same bits) rather than read
      // from another workgroup's memory
      make_hypothesis(a.corr, a.ld, base, n, a.k0, a.k1, hyp, static_cast<uint32_t>(p), bestH);
      a.best_count[p] = static_cast<int32_t>(key_count(key));
      a.best_hyp[p] = static_cast<int32_t>(hyp);
    } else {
#pragma unroll
      for (int k = 0; k < 9; ++k) bestH[k] = 0.0f;
      a.best_count[p] = 0;
      a.best_hyp[p] = -1;
    }
    skey = key;
  }
  __syncthreads();
  if (threadIdx.x < 9) a.best_H[9 * p + threadIdx.x] = bestH[threadIdx.x];
  const bool any = skey != 0ull;
  double hh[9];
#pragma unroll
  for (int k = 0; k < 9; ++k) hh[k] = bestH[k];
  const float *X1 = a.corr + base, *Y1 = a.corr + a.ld + base;
  const float *X2 = a.corr + 2 * a.ld + base, *Y2 = a.corr + 3 * a.ld + base;
  // 4 points per thread in flight (indices clamped into the pair for the loads)
  for (uint32_t i0 = threadIdx.x; i0 < n; i0 += 4u * kFinishThreads) {
    float x1[4], y1[4], x2[4], y2[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const uint32_t j = min(i0 + static_cast<uint32_t>(u) * kFinishThreads, n - 1u);
      x1[u] = X1[j];
      y1[u] = Y1[j];
      x2[u] = X2[j];
      y2[u] = Y2[j];
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const uint32_t i = i0 + static_cast<uint32_t>(u) * kFinishThreads;
      if (i < n)
        a.mask[base + i] = (any && inlier_f64(hh, x1[u], y1[u], x2[u], y2[u], a.tau)) ? 1 : 0;
    }
  }
}

// Single pair, after the fused kernel: reduce the work items' best keys (every
// workgroup does it redundantly), then write the best outputs (workgroup 0)
// and this workgroup's slice of the inlier mask.
__global__ __launch_bounds__(kThreads) void ransac_mask_kernel(RansacArgs a) {
  __shared__ unsigned long long red[kWaves];
  __shared__ float bh[9];
  unsigned long long best = 0ull;
  for (int64_t j = threadIdx.x; j < a.n_items; j += kThreads) best = max(best, a.blockbest[j]);
  best = wave_max_u64(best);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = best;
  __syncthreads();
  unsigned long long key = 0ull;
#pragma unroll
  for (int w = 0; w < kWaves; ++w) key = max(key, red[w]);
  const bool any = key != 0ull;
  const uint32_t hyp = any ? 0xFFFFFFFFu - static_cast<uint32_t>(key & 0xFFFFFFFFull) : 0u;
  if (threadIdx.x < 9) bh[threadIdx.x] = any ? a.hbuf[9ull * hyp + threadIdx.x] : 0.0f;
  __syncthreads();
  if (blockIdx.x == 0 && threadIdx.x < 9) a.best_H[threadIdx.x] = bh[threadIdx.x];
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    a.best_count[0] = any ? static_cast<int32_t>((key >> 32) - 1ull) : 0;
    a.best_hyp[0] = any ? static_cast<int32_t>(hyp) : -1;
  }
  double hh[9];
#pragma unroll
  for (int k = 0; k < 9; ++k) hh[k] = bh[k];
  const int n = a.n_single;
  const float *X1 = a.corr, *Y1 = a.corr + a.ld, *X2 = a.corr + 2 * a.ld, *Y2 = a.corr + 3 * a.ld;
  for (int i = blockIdx.x * kThreads + threadIdx.x; i < n; i += gridDim.x * kThreads)
    a.mask[i] = (any && inlier_f64(hh, X1[i], Y1[i], X2[i], Y2[i], a.tau)) ? 1 : 0;
}

// Resets keys, the queue and the adaptive state, and ranks pairs by size (largest
// first, ties by index). Pair q's sort key is (N_q << 32) | ~q, unique per
// pair, so the rank of p (the number of larger keys) is a permutation of
// 0 .. n_pairs - 1. One wave ranks one pair; the keys are staged through LDS
// in tiles of kThreads, shared by the workgroup's waves. Launched with one
// wave per pair (at least one workgroup).
__global__ __launch_bounds__(kThreads) void ransac_prep_kernel(RansacArgs a, int rank) {
  __shared__ unsigned long long tile[kThreads];
  const int64_t g = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  const int64_t stride = static_cast<int64_t>(gridDim.x) * blockDim.x;
  if (g == 0 && a.queue) *a.queue = 0u;
  for (int64_t q = g; q < a.n_pairs; q += stride) {
    if (a.keys) a.keys[q] = 0ull;
    if (a.pst) {
      a.pst[q].prefix = 0ull;
      a.pst[q].stop = static_cast<uint32_t>(a.n_hb);
      a.pst[q].pad = 0u;
    }
  }
  if (a.rkey) {
    const int64_t total = static_cast<int64_t>(a.n_pairs) * a.n_hb;
    for (int64_t i = g; i < total; i += stride) a.rkey[i] = kUnpublished;
  }
  if (!a.order) return;
  int32_t *order = const_cast<int32_t *>(a.order);
  if (!rank) {
    for (int64_t q = g; q < a.n_pairs; q += stride) order[q] = static_cast<int32_t>(q);
    return;
  }
  auto sort_key = [&](int q) {
    int64_t b;
    uint32_t n = 0u;
    pair_range(a, q, b, n);
    return (static_cast<unsigned long long>(n) << 32) | (0xFFFFFFFFu - static_cast<uint32_t>(q));
  };
  const int p = static_cast<int>(g >> 6);   // this wave's pair (uniform across the wave)
  const int lane = threadIdx.x & 63;
  const unsigned long long kp = p < a.n_pairs ? sort_key(p) : ~0ull;
  int r = 0;
  for (int q0 = 0; q0 < a.n_pairs; q0 += kThreads) {
    const int q = q0 + threadIdx.x;
    __syncthreads();
    tile[threadIdx.x] = q < a.n_pairs ? sort_key(q) : 0ull;   // 0: below every real key
    __syncthreads();
    for (int k = lane; k < kThreads; k += 64) r += tile[k] > kp ? 1 : 0;
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) r += __shfl_xor(r, o);
  if (p < a.n_pairs && lane == 0) order[r] = p;
}

// Queue order of the adaptive rounds. Round r of pair p is placed by
// (2r + 1) / N_p, the midpoint of that round on a clock where each of the
// pair's rounds takes N_p units (ties: lower pair index first). The rounds of
// a large pair are spread over the queue instead of being stacked at its end,
// so that the last items are rounds of small pairs; rounds of small pairs
// come later than under plain round order, when more stopping points are
// known. One wave per item: its position is the number of items placed before
// it, counted exactly in integers over all pairs.
__global__ __launch_bounds__(kThreads) void ransac_round_order_kernel(RansacArgs a) {
  __shared__ int64_t nsz[kThreads];
  const int64_t item = (static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x) >> 6;
  const int lane = threadIdx.x & 63;
  const int64_t total = static_cast<int64_t>(a.n_pairs) * a.n_hb;
  const bool live = item < total;   // uniform across the wave
  const int p = live ? static_cast<int>(item / a.n_hb) : 0;
  const int64_t r = live ? item % a.n_hb : 0;
  int64_t b;
  uint32_t n;
  pair_range(a, p, b, n);
  const int64_t np = max(n, 1u);
  const double inv = 1.0 / static_cast<double>(np);
  const int64_t R = a.n_hb;
  const int64_t cap = (2 * R + 2) * np;   // x >= cap: every round of q comes first
  int64_t pos = 0;
  // pair sizes staged through LDS, kThreads at a time, shared by the workgroup's waves
  for (int q0 = 0; q0 < a.n_pairs; q0 += kThreads) {
    __syncthreads();
    if (q0 + static_cast<int>(threadIdx.x) < a.n_pairs) {
      pair_range(a, q0 + threadIdx.x, b, n);
      nsz[threadIdx.x] = max(n, 1u);
    }
    __syncthreads();
    const int qn = min(kThreads, a.n_pairs - q0);
    for (int k = lane; k < qn; k += 64) {
      const int64_t x = (2 * r + 1) * nsz[k];
      if (x >= cap) {
        pos += R;
        continue;
      }
      // c = ceil(x / np): the double estimate is within one of it (x / np < 2R + 2),
      // and one exact integer step corrects it
      int64_t c = static_cast<int64_t>(ceil(static_cast<double>(x) * inv));
      if ((c - 1) * np >= x)
        --c;
      else if (c * np < x)
        ++c;
      // rounds r' of pair q with (2r' + 1) / N_q < (2r + 1) / N_p: the odd numbers below x / np
      pos += min(R, c / 2);
      // equal position: the round (c - 1) / 2 of a lower-numbered pair goes first
      if (q0 + k < p && c * np == x && (c & 1) && (c - 1) / 2 < R) pos += 1;
    }
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) pos += __shfl_xor(pos, o);
  if (live && lane == 0 && pos >= 0 && pos < total)
    a.iorder[pos] = static_cast<int32_t>(static_cast<int64_t>(p) * a.n_hb + r);
}

// ---- plain single-pair form -------------------------------------------------

__global__ void plain_solve_kernel(RansacArgs a, float *Hbuf, uint32_t *valid) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= a.n_hyp) return;
  float h[9];
  const uint32_t f = make_hypothesis(a.corr, a.ld, 0, static_cast<uint32_t>(a.n_single), a.k0,
                                     a.k1, static_cast<uint32_t>(j), 0u, h);
#pragma unroll
  for (int k = 0; k < 9; ++k) Hbuf[9 * j + k] = h[k];
  valid[j] = f == 0u ? 1u : 0u;
}

template <int P, int HB>
__global__ __launch_bounds__(kThreads) void plain_score_kernel(RansacArgs a, const float *Hbuf,
                                                               const uint32_t *valid,
                                                               int32_t *counts) {
  __shared__ float Hs[HB][9];
  __shared__ double H0s[HB][9];
  __shared__ uint32_t vs[HB];
  __shared__ uint32_t cnt[HB];
  __shared__ FixList fix;
  __shared__ uint32_t ub[HB];
  const int h0 = blockIdx.x * HB;
  const int nh = min(HB, a.n_hyp - h0);
  for (int i = threadIdx.x; i < HB * 9; i += kThreads) {
    const float v = (i / 9 < nh) ? Hbuf[9 * h0 + i] : 0.0f;
    Hs[i / 9][i % 9] = (i % 9 < 6) ? v * a.inv_tau : v;   // scoring form
    H0s[i / 9][i % 9] = v;
  }
  for (int i = threadIdx.x; i < HB; i += kThreads) {
    vs[i] = (i < nh) ? valid[h0 + i] : 0u;
    cnt[i] = 0u;
  }
  if (threadIdx.x == 0) fix.n = 0u;
  __syncthreads();
  const int lane = threadIdx.x & 63;
  const uint64_t vmask = __ballot(lane < nh && vs[lane] != 0u);
  score_hyps<P>(a, 0, static_cast<uint32_t>(a.n_single), Hs, vmask, nh, cnt, &fix);
  __syncthreads();
  fix_counts<kWaves>(a, 0, static_cast<uint32_t>(a.n_single), H0s, &fix, vmask, nh, cnt,
             a.hyp_counts != nullptr, ub);
  if (threadIdx.x < nh)
    counts[h0 + threadIdx.x] = vs[threadIdx.x] ? static_cast<int32_t>(cnt[threadIdx.x]) : -1;
}

// One workgroup: argmax over counts (-1 = invalid), ties to the lower index.
constexpr int kArgmaxThreads = 1024;
__global__ __launch_bounds__(kArgmaxThreads) void plain_argmax_kernel(const int32_t *counts,
                                                                      int n_hyp,
                                                                      unsigned long long *key,
                                                                      int32_t *hyp_counts) {
  __shared__ unsigned long long red[kArgmaxThreads / 64];
  unsigned long long best = 0ull;
  for (int j = threadIdx.x; j < n_hyp; j += kArgmaxThreads) {
    const int32_t c = counts[j];
    if (hyp_counts) hyp_counts[j] = c < 0 ? 0 : c;
    if (c >= 0) best = max(best, pack_key(static_cast<uint32_t>(c), static_cast<uint32_t>(j)));
  }
  best = wave_max_u64(best);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = best;
  __syncthreads();
  if (threadIdx.x < 64) {
    unsigned long long v = threadIdx.x < kArgmaxThreads / 64 ? red[threadIdx.x] : 0ull;
    v = wave_max_u64(v);
    if (threadIdx.x == 0) *key = v;
  }
}

__global__ __launch_bounds__(kThreads) void plain_mask_kernel(RansacArgs a, const float *Hbuf,
                                                              const unsigned long long *key) {
  const unsigned long long k = *key;
  const bool any = k != 0ull;
  const uint32_t hyp = any ? 0xFFFFFFFFu - static_cast<uint32_t>(k & 0xFFFFFFFFull) : 0u;
  float bh[9];
  double bd[9];
#pragma unroll
  for (int i = 0; i < 9; ++i) {
    bh[i] = any ? Hbuf[9 * hyp + i] : 0.0f;
    bd[i] = bh[i];
  }
  if (blockIdx.x == 0 && threadIdx.x < 9) a.best_H[threadIdx.x] = bh[threadIdx.x];
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    a.best_count[0] = any ? static_cast<int32_t>((k >> 32) - 1ull) : 0;
    a.best_hyp[0] = any ? static_cast<int32_t>(hyp) : -1;
  }
  const int n = a.n_single;
  const float *X1 = a.corr, *Y1 = a.corr + a.ld, *X2 = a.corr + 2 * a.ld, *Y2 = a.corr + 3 * a.ld;
  for (int i = blockIdx.x * kThreads + threadIdx.x; i < n; i += gridDim.x * kThreads)
    a.mask[i] = (any && inlier_f64(bd, X1[i], Y1[i], X2[i], Y2[i], a.tau)) ? 1 : 0;
}

// ---- tuning --------------------------------------------------------------

struct Tune {
  int P, HB, bpc;
};

static bool tune_valid(const hg_ransac_tuning &t) {
  return (t.pts_per_lane == 8 || t.pts_per_lane == 16) &&
         (t.hyps_per_block == 16 || t.hyps_per_block == 32 || t.hyps_per_block == 64) &&
         t.blocks_per_cu >= 1 && t.blocks_per_cu <= 8;
}

static const hg_ransac_tuning kDefaultTune = {16, 64, 4, 0};

typedef void (*KernelFn)(RansacArgs);

template <bool PERSISTENT>
static KernelFn pick_kernel(int P, int HB) {
#define HG_PICK(PP, HH) \
  if (P == PP && HB == HH) return ransac_kernel<PP, HH, PERSISTENT>;
  HG_PICK(8, 4) HG_PICK(8, 8) HG_PICK(8, 16) HG_PICK(8, 32) HG_PICK(8, 64)
  HG_PICK(16, 16) HG_PICK(16, 32) HG_PICK(16, 64)
#undef HG_PICK
  return nullptr;
}

static std::mutex g_tune_mu;
static std::map<std::string, hg_ransac_tuning> g_tune_cache;
static bool g_tune_file_read = false;

static std::string tune_key(int n_pairs, int n_hyp) {
  int dev = 0;
  (void)hipGetDevice(&dev);
  char buf[128];
  snprintf(buf, sizeof buf, "gfx950:%d:%d:%d", device_cus(), n_pairs, n_hyp);
  return buf;
}

static void read_tune_file() {
  if (g_tune_file_read) return;
  g_tune_file_read = true;
  const char *path = getenv("HG_AUTOTUNE_CACHE");
  if (!path) return;
  FILE *f = fopen(path, "r");
  if (!f) return;
  char line[512];
  while (fgets(line, sizeof line, f)) {
    char key[256];
    hg_ransac_tuning t = {0, 0, 0, 0};
    if (sscanf(line, " \"%255[^\"]\" : [ %d , %d , %d ]", key, &t.pts_per_lane,
               &t.hyps_per_block, &t.blocks_per_cu) == 4 &&
        tune_valid(t))
      g_tune_cache[key] = t;
  }
  fclose(f);
}

static void write_tune_file() {
  const char *path = getenv("HG_AUTOTUNE_CACHE");
  if (!path) return;
  FILE *f = fopen(path, "w");
  if (!f) return;
  fprintf(f, "{\n");
  size_t i = 0;
  for (const auto &kv : g_tune_cache) {
    fprintf(f, "  \"%s\": [%d, %d, %d]%s\n", kv.first.c_str(), kv.second.pts_per_lane,
            kv.second.hyps_per_block, kv.second.blocks_per_cu,
            ++i < g_tune_cache.size() ? "," : "");
  }
  fprintf(f, "}\n");
  fclose(f);
}

static hg_ransac_tuning lookup_tune(int n_pairs, int n_hyp) {
  std::lock_guard<std::mutex> lock(g_tune_mu);
  read_tune_file();
  auto it = g_tune_cache.find(tune_key(n_pairs, n_hyp));
  return it == g_tune_cache.end() ? kDefaultTune : it->second;
}

// ---- workspace layout ------------------------------------------------------

static size_t align256(size_t x) { return (x + 255) & ~static_cast<size_t>(255); }

struct BatchedWs {
  unsigned long long *keys;
  int32_t *order;
  uint32_t *queue;
};

static size_t batched_ws_bytes(int n_pairs) {
  return align256(8ull * n_pairs) + align256(4ull * n_pairs) + 256;
}

static BatchedWs carve_batched(void *ws, int n_pairs) {
  char *p = static_cast<char *>(ws);
  BatchedWs w;
  w.keys = reinterpret_cast<unsigned long long *>(p);
  p += align256(8ull * n_pairs);
  w.order = reinterpret_cast<int32_t *>(p);
  p += align256(4ull * n_pairs);
  w.queue = reinterpret_cast<uint32_t *>(p);
  return w;
}

static size_t plain_ws_bytes(int n_hyp) {
  return align256(36ull * n_hyp) + align256(4ull * n_hyp) + align256(4ull * n_hyp) + 256;
}

// ---- host launchers --------------------------------------------------------

static int check_single(const float *corr, int32_t n_pts, int64_t ld, int32_t n_hyp, float thresh,
                        float *best_H, int32_t *best_count, int32_t *best_hyp, uint8_t *mask,
                        void *ws, size_t ws_bytes, size_t need) {
  HG_REQUIRE(corr && best_H && best_count && best_hyp && mask,
             "hg_ransac: NULL corr or output pointer");
  HG_REQUIRE(n_pts >= 4, "hg_ransac: n_pts = %d < 4", n_pts);
  HG_REQUIRE(ld >= n_pts, "hg_ransac: ld < n_pts");
  HG_REQUIRE(n_hyp >= 1, "hg_ransac: n_hyp = %d < 1", n_hyp);
  HG_REQUIRE(std::isfinite(thresh) && thresh > 0.0f && std::isfinite(1.0f / thresh),
             "hg_ransac: threshold must be finite and > 0 (and 1/threshold finite)");
  if (!ws || ws_bytes < need)
    return fail(HG_EWORKSPACE, "hg_ransac: workspace of %zu bytes needed, %zu given", need,
                ws ? ws_bytes : static_cast<size_t>(0));
  HG_REQUIRE(aligned(ws, 256), "hg_ransac: workspace must be 256-byte aligned");
  return HG_OK;
}

static RansacArgs make_args(const float *corr, int64_t ld, const int64_t *off, int32_t n_single,
                            int32_t n_pairs, int32_t n_hyp, int HB, float thresh, uint64_t seed,
                            float *best_H, int32_t *best_count, int32_t *best_hyp, uint8_t *mask,
                            int32_t *hyp_counts) {
  RansacArgs a;
  a.corr = corr;
  a.ld = ld;
  a.off = off;
  a.n_single = n_single;
  a.n_pairs = n_pairs;
  a.n_hyp = n_hyp;
  a.n_hb = (n_hyp + HB - 1) / HB;
  a.n_items = static_cast<int64_t>(n_pairs) * a.n_hb;
  a.tau = thresh;
  a.inv_tau = 1.0f / thresh;
  a.k0 = static_cast<uint32_t>(seed & 0xFFFFFFFFull);
  a.k1 = static_cast<uint32_t>(seed >> 32);
  a.best_H = best_H;
  a.best_count = best_count;
  a.best_hyp = best_hyp;
  a.mask = mask;
  a.hyp_counts = hyp_counts;
  a.keys = nullptr;
  a.queue = nullptr;
  a.order = nullptr;
  a.hbuf = nullptr;
  a.blockbest = nullptr;
  a.pst = nullptr;
  a.rkey = nullptr;
  a.iorder = nullptr;
  a.n_eval = nullptr;
  a.one_minus_conf = 0.0;
  return a;
}

// Enqueue the batched form (prep, round order, persistent kernel, finish) on
// stream s.
static int launch_batched(const RansacArgs &a0, const hg_ransac_tuning &t, void *ws,
                          hipStream_t s) {
  RansacArgs a = a0;
  const BatchedWs w = carve_batched(ws, a.n_pairs);
  a.keys = w.keys;
  a.queue = w.queue;
  a.order = w.order;
  const int rank = a.n_pairs <= 65536 ? 1 : 0;
  // one wave per pair when ranking (ranks of 65536 pairs: 16384 workgroups)
  const int64_t prep_blocks = rank ? (static_cast<int64_t>(a.n_pairs) + kWaves - 1) / kWaves
                                   : (static_cast<int64_t>(a.n_pairs) + kThreads - 1) / kThreads;
  hipLaunchKernelGGL(ransac_prep_kernel, dim3(static_cast<unsigned>(prep_blocks)),
                     dim3(kThreads), 0, s, a, rank);
  if (int st = launched("ransac_prep_kernel")) return st;
  if (a.iorder) {
    const int64_t waves = static_cast<int64_t>(a.n_pairs) * a.n_hb;
    const int64_t blocks = (waves + kWaves - 1) / kWaves;
    hipLaunchKernelGGL(ransac_round_order_kernel, dim3(static_cast<unsigned>(blocks)),
                       dim3(kThreads), 0, s, a);
    if (int st = launched("ransac_round_order_kernel")) return st;
  }
  KernelFn k = pick_kernel<true>(t.pts_per_lane, t.hyps_per_block);
  if (!k) return fail(HG_EINVAL, "unsupported tuning");
  const int64_t blocks = std::min<int64_t>(static_cast<int64_t>(device_cus()) * t.blocks_per_cu,
                                           std::max<int64_t>(1, a.n_items));
  hipLaunchKernelGGL(k, dim3(static_cast<unsigned>(blocks)), dim3(kThreads), 0, s, a);
  if (int st = launched("ransac_kernel<persistent>")) return st;
  hipLaunchKernelGGL(ransac_finish_kernel, dim3(static_cast<unsigned>(a.n_pairs)),
                     dim3(kFinishThreads), 0, s, a);
  return launched("ransac_finish_kernel");
}

static int check_batched(const float *corr, int64_t ld, const int64_t *off, int32_t n_pairs,
                         int32_t n_hyp, float thresh, const hg_ransac_tuning *tune, float *best_H,
                         int32_t *best_count, int32_t *best_hyp, uint8_t *mask, void *ws,
                         size_t ws_bytes) {
  HG_REQUIRE(corr && off && best_H && best_count && best_hyp && mask,
             "hg_ransac_batched: NULL corr, off or output pointer");
  HG_REQUIRE(n_pairs >= 1, "hg_ransac_batched: n_pairs = %d < 1", n_pairs);
  HG_REQUIRE(ld >= 1, "hg_ransac_batched: ld < 1");
  HG_REQUIRE(n_hyp >= 1, "hg_ransac_batched: n_hyp = %d < 1", n_hyp);
  // the persistent queue is a 32-bit counter that every workgroup also bumps
  // once past the end: at most 2^31 work items (of >= 16 hypotheses) keep it
  // from wrapping, which would restart the queue and never end the launch
  HG_REQUIRE(static_cast<int64_t>(n_pairs) * ((static_cast<int64_t>(n_hyp) + 15) / 16) <=
                 (int64_t(1) << 31),
             "hg_ransac_batched: n_pairs x n_hyp too large for one launch (n_pairs * "
             "ceil(n_hyp / 16) must be <= 2^31)");
  HG_REQUIRE(std::isfinite(thresh) && thresh > 0.0f && std::isfinite(1.0f / thresh),
             "hg_ransac_batched: threshold must be finite and > 0 (and 1/threshold finite)");
  HG_REQUIRE(!tune || tune_valid(*tune), "hg_ransac_batched: unsupported tuning");
  const size_t need = batched_ws_bytes(n_pairs);
  if (!ws || ws_bytes < need)
    return fail(HG_EWORKSPACE, "hg_ransac_batched: workspace of %zu bytes needed, %zu given",
                need, ws ? ws_bytes : static_cast<size_t>(0));
  HG_REQUIRE(aligned(ws, 256), "hg_ransac_batched: workspace must be 256-byte aligned");
  return HG_OK;
}

}  // namespace hg

using namespace hg;

namespace hg {

// Workspace of the fused single-pair form: every hypothesis's H and each work
// item's best key (at least 4 hypotheses per item).
static size_t fused_ws_bytes(int32_t n_hyp) {
  return align256(36ull * n_hyp) + align256(8ull * ((n_hyp + 3) / 4));
}

// Enqueue the fused single-pair form (scoring kernel + mask kernel) with
// workspace ws (validated by the caller).
static int launch_fused(const float *corr, int32_t n_pts, int64_t ld, int32_t n_hyp, float thresh,
                        uint64_t seed, float *best_H, int32_t *best_count, int32_t *best_hyp,
                        uint8_t *inlier_mask, int32_t *hyp_counts, void *ws, hipStream_t s) {
  // about two workgroups per compute unit when the hypothesis count allows it
  int HB = 4;
  while (HB < 64 && static_cast<int64_t>(HB) * 2 * device_cus() < n_hyp) HB *= 2;
  const int P = 8;
  RansacArgs a = make_args(corr, ld, nullptr, n_pts, 1, n_hyp, HB, thresh, seed, best_H,
                           best_count, best_hyp, inlier_mask, hyp_counts);
  char *w = static_cast<char *>(ws);
  a.hbuf = reinterpret_cast<float *>(w);
  a.blockbest = reinterpret_cast<unsigned long long *>(w + align256(36ull * n_hyp));
  KernelFn k = pick_kernel<false>(P, HB);
  hipLaunchKernelGGL(k, dim3(static_cast<unsigned>(a.n_items)), dim3(kFusedWaves * 64), 0, s, a);
  if (int st = launched("ransac_kernel<fused>")) return st;
  const int mb = std::max(1, std::min(1024, (n_pts + kThreads - 1) / kThreads));
  hipLaunchKernelGGL(ransac_mask_kernel, dim3(mb), dim3(kThreads), 0, s, a);
  return launched("ransac_mask_kernel");
}

// The library's own workspace for hg_ransac_noalloc: a static device array
// (each GPU the library runs on holds its own copy until the process ends).
// Host code never uses this name as an address: the device address is looked
// up once per device (hipGetSymbolAddress) and kept in g_noalloc_ws.
constexpr int32_t kNoAllocMaxHyp = 16384;
constexpr size_t kNoAllocBytes = 36ull * kNoAllocMaxHyp + 8ull * (kNoAllocMaxHyp / 4);
static_assert(kNoAllocBytes % 256 == 0, "whole 256-byte blocks");
static __device__ __align__(256) unsigned char scratch[kNoAllocBytes];

static std::mutex g_noalloc_mu;
static void *g_noalloc_ws[64] = {nullptr};

// Device address of `scratch` on the current device (looked up on the first
// call on each device, with that device current).
static int noalloc_ws(void **out) {
  int dev = 0;
  HG_HIP(hipGetDevice(&dev));
  HG_REQUIRE(dev >= 0 && dev < 64, "hg_ransac_noalloc: device ordinal %d out of range", dev);
  std::lock_guard<std::mutex> lock(g_noalloc_mu);
  if (!g_noalloc_ws[dev]) {
    void *ptr = nullptr;
    HG_HIP(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
    HG_REQUIRE(ptr != nullptr && aligned(ptr, 256), "hg_ransac_noalloc: bad workspace address");
    g_noalloc_ws[dev] = ptr;
  }
  *out = g_noalloc_ws[dev];
  return HG_OK;
}

}  // namespace hg

extern "C" size_t hg_ransac_ws_bytes(int32_t n_pts, int32_t n_hyp) {
  (void)n_pts;
  if (n_hyp < 1) n_hyp = 1;
  // fused: H of every hypothesis and per-item best keys; plain: H buffer,
  // validity, counts and the argmax key
  return std::max(fused_ws_bytes(n_hyp), plain_ws_bytes(n_hyp));
}

extern "C" int hg_ransac(const float *corr, int32_t n_pts, int64_t ld, int32_t n_hyp,
                         float thresh, uint64_t seed, float *best_H, int32_t *best_count,
                         int32_t *best_hyp, uint8_t *inlier_mask, int32_t *hyp_counts, void *ws,
                         size_t ws_bytes, void *stream) {
  clear_error();
  if (int st = check_single(corr, n_pts, ld, n_hyp, thresh, best_H, best_count, best_hyp,
                            inlier_mask, ws, ws_bytes, hg_ransac_ws_bytes(n_pts, n_hyp)))
    return st;
  return launch_fused(corr, n_pts, ld, n_hyp, thresh, seed, best_H, best_count, best_hyp,
                      inlier_mask, hyp_counts, ws, as_stream(stream));
}

extern "C" int hg_ransac_noalloc(const float *corr, int32_t n_pts, int64_t ld, int32_t n_hyp,
                                 float thresh, uint64_t seed, float *best_H, int32_t *best_count,
                                 int32_t *best_hyp, uint8_t *inlier_mask, int32_t *hyp_counts,
                                 void *stream) {
  clear_error();
  HG_REQUIRE(n_hyp <= kNoAllocMaxHyp,
             "hg_ransac_noalloc: n_hyp = %d exceeds the maximum of %d (use hg_ransac with a "
             "caller workspace)", n_hyp, kNoAllocMaxHyp);
  // arguments first (host only; any aligned non-null address stands for the
  // workspace here), then the workspace's device address
  if (int st = check_single(corr, n_pts, ld, n_hyp, thresh, best_H, best_count, best_hyp,
                            inlier_mask, reinterpret_cast<void *>(256), kNoAllocBytes,
                            fused_ws_bytes(n_hyp)))
    return st;
  void *ws = nullptr;
  if (int st = noalloc_ws(&ws)) return st;
  return launch_fused(corr, n_pts, ld, n_hyp, thresh, seed, best_H, best_count, best_hyp,
                      inlier_mask, hyp_counts, ws, as_stream(stream));
}

extern "C" int hg_ransac_plain(const float *corr, int32_t n_pts, int64_t ld, int32_t n_hyp,
                               float thresh, uint64_t seed, float *best_H, int32_t *best_count,
                               int32_t *best_hyp, uint8_t *inlier_mask, int32_t *hyp_counts,
                               void *ws, size_t ws_bytes, void *stream) {
  clear_error();
  if (int st = check_single(corr, n_pts, ld, n_hyp, thresh, best_H, best_count, best_hyp,
                            inlier_mask, ws, ws_bytes, hg_ransac_ws_bytes(n_pts, n_hyp)))
    return st;
  const hipStream_t s = as_stream(stream);
  constexpr int HB = 16, P = 8;
  RansacArgs a = make_args(corr, ld, nullptr, n_pts, 1, n_hyp, HB, thresh, seed, best_H,
                           best_count, best_hyp, inlier_mask, hyp_counts);
  char *p = static_cast<char *>(ws);
  float *Hbuf = reinterpret_cast<float *>(p);
  p += align256(36ull * n_hyp);
  uint32_t *valid = reinterpret_cast<uint32_t *>(p);
  p += align256(4ull * n_hyp);
  int32_t *counts = reinterpret_cast<int32_t *>(p);
  p += align256(4ull * n_hyp);
  unsigned long long *key = reinterpret_cast<unsigned long long *>(p);
  hipLaunchKernelGGL(plain_solve_kernel, dim3((n_hyp + 255) / 256), dim3(256), 0, s, a, Hbuf,
                     valid);
  if (int st = launched("plain_solve_kernel")) return st;
  hipLaunchKernelGGL((plain_score_kernel<P, HB>), dim3((n_hyp + HB - 1) / HB), dim3(kThreads), 0,
                     s, a, Hbuf, valid, counts);
  if (int st = launched("plain_score_kernel")) return st;
  hipLaunchKernelGGL(plain_argmax_kernel, dim3(1), dim3(kArgmaxThreads), 0, s, counts, n_hyp, key,
                     hyp_counts);
  if (int st = launched("plain_argmax_kernel")) return st;
  const int mb = std::max(1, std::min(1024, (n_pts + kThreads - 1) / kThreads));
  hipLaunchKernelGGL(plain_mask_kernel, dim3(mb), dim3(kThreads), 0, s, a, Hbuf, key);
  return launched("plain_mask_kernel");
}

extern "C" size_t hg_ransac_batched_ws_bytes(int32_t n_pairs, int32_t n_hyp) {
  (void)n_hyp;
  return batched_ws_bytes(n_pairs < 1 ? 1 : n_pairs);
}

extern "C" int hg_ransac_batched(const float *corr, int64_t ld, const int64_t *off,
                                 int32_t n_pairs, int32_t n_hyp, float thresh, uint64_t seed,
                                 const hg_ransac_tuning *tune, float *best_H, int32_t *best_count,
                                 int32_t *best_hyp, uint8_t *inlier_mask, int32_t *hyp_counts,
                                 void *ws, size_t ws_bytes, void *stream) {
  clear_error();
  if (int st = check_batched(corr, ld, off, n_pairs, n_hyp, thresh, tune, best_H, best_count,
                             best_hyp, inlier_mask, ws, ws_bytes))
    return st;
  const hg_ransac_tuning t = tune ? *tune : lookup_tune(n_pairs, n_hyp);
  RansacArgs a = make_args(corr, ld, off, 0, n_pairs, n_hyp, t.hyps_per_block, thresh, seed,
                           best_H, best_count, best_hyp, inlier_mask, hyp_counts);
  return launch_batched(a, t, ws, as_stream(stream));
}

extern "C" int hg_ransac_autotune(const float *corr, int64_t ld, const int64_t *off,
                                  const int64_t *off_host, int32_t n_pairs, int32_t n_hyp,
                                  float thresh, uint64_t seed, void *ws, size_t ws_bytes,
                                  void *stream, hg_ransac_tuning *out) {
  clear_error();
  HG_REQUIRE(off_host && out, "hg_ransac_autotune: NULL off_host or out");
  HG_REQUIRE(n_pairs >= 1, "hg_ransac_autotune: n_pairs < 1");
  const int64_t total = off_host[n_pairs];
  HG_REQUIRE(total >= 0 && ld >= total, "hg_ransac_autotune: ld < total points");
  float *bh = nullptr;
  int32_t *bc = nullptr, *bi = nullptr;
  uint8_t *mk = nullptr;
  // validate with dummy output pointers first (host only)
  if (int st = check_batched(corr, ld, off, n_pairs, n_hyp, thresh, nullptr,
                             reinterpret_cast<float *>(1), reinterpret_cast<int32_t *>(1),
                             reinterpret_cast<int32_t *>(1), reinterpret_cast<uint8_t *>(1), ws,
                             ws_bytes))
    return st;
  const hipStream_t s = as_stream(stream);
  hipEvent_t e0 = nullptr, e1 = nullptr;
  // frees whatever was obtained, on every return path
  struct Scratch {
    float **bh;
    int32_t **bc, **bi;
    uint8_t **mk;
    hipEvent_t *e0, *e1;
    ~Scratch() {
      if (*e0) (void)hipEventDestroy(*e0);
      if (*e1) (void)hipEventDestroy(*e1);
      if (*bh) (void)hipFree(*bh);
      if (*bc) (void)hipFree(*bc);
      if (*bi) (void)hipFree(*bi);
      if (*mk) (void)hipFree(*mk);
    }
  } scratch{&bh, &bc, &bi, &mk, &e0, &e1};
  HG_HIP(hipMalloc(&bh, 36ull * n_pairs));
  HG_HIP(hipMalloc(&bc, 4ull * n_pairs));
  HG_HIP(hipMalloc(&bi, 4ull * n_pairs));
  // the kernels clamp pair ranges into [0, ld), so a mask of ld bytes covers any offsets
  HG_HIP(hipMalloc(&mk, static_cast<size_t>(std::max<int64_t>(ld, 1))));
  HG_HIP(hipEventCreate(&e0));
  HG_HIP(hipEventCreate(&e1));
  float best_ms = 1e30f;
  hg_ransac_tuning best = kDefaultTune;
  int status = HG_OK;
  for (int P : {8, 16})
    for (int HB : {16, 32, 64})
      for (int bpc : {1, 2, 4, 5, 6}) {
        const hg_ransac_tuning t = {P, HB, bpc, 0};
        RansacArgs a = make_args(corr, ld, off, 0, n_pairs, n_hyp, HB, thresh, seed, bh, bc, bi,
                                 mk, nullptr);
        if ((status = launch_batched(a, t, ws, s)) != HG_OK) goto done;   // warm-up
        float ms[3];
        for (int r = 0; r < 3; ++r) {
          (void)hipEventRecord(e0, s);
          if ((status = launch_batched(a, t, ws, s)) != HG_OK) goto done;
          (void)hipEventRecord(e1, s);
          if (hipEventSynchronize(e1) != hipSuccess) {
            status = fail(HG_EHIP, "autotune: event sync failed");
            goto done;
          }
          (void)hipEventElapsedTime(&ms[r], e0, e1);
        }
        std::sort(ms, ms + 3);
        if (ms[1] < best_ms) {
          best_ms = ms[1];
          best = t;
        }
      }
done:
  (void)hipStreamSynchronize(s);   // the scratch buffers are released when this returns
  if (status != HG_OK) return status;
  *out = best;
  {
    std::lock_guard<std::mutex> lock(g_tune_mu);
    read_tune_file();
    g_tune_cache[tune_key(n_pairs, n_hyp)] = best;
    write_tune_file();
  }
  return HG_OK;
}

// ---- adaptive termination ---------------------------------------------------

constexpr int kRound = kRoundHyps;

static size_t adaptive_extra_bytes(int n_pairs, int n_hyp) {
  const int64_t nr = (static_cast<int64_t>(n_hyp) + kRound - 1) / kRound;
  return align256(sizeof(PairState) * static_cast<size_t>(n_pairs)) +
         align256(8ull * n_pairs * nr) + align256(4ull * n_pairs * nr);
}

// The staggered round order costs n_pairs^2 * rounds integer steps: used up
// to 2^27 of them (e.g. 2048 pairs of 1024 hypotheses), round order beyond.
static bool stagger_rounds(int64_t n_pairs, int64_t n_rounds) {
  return n_pairs * n_pairs * n_rounds <= (int64_t(1) << 27);
}

extern "C" size_t hg_ransac_adaptive_ws_bytes(int32_t n_pairs, int32_t n_hyp_max) {
  if (n_pairs < 1) n_pairs = 1;
  if (n_hyp_max < 1) n_hyp_max = 1;
  return batched_ws_bytes(n_pairs) + adaptive_extra_bytes(n_pairs, n_hyp_max);
}

extern "C" int hg_ransac_adaptive(const float *corr, int64_t ld, const int64_t *off,
                                  int32_t n_pairs, int32_t n_hyp_max, float thresh, uint64_t seed,
                                  double confidence, const hg_ransac_tuning *tune, float *best_H,
                                  int32_t *best_count, int32_t *best_hyp, uint8_t *inlier_mask,
                                  int32_t *n_evaluated, void *ws, size_t ws_bytes, void *stream) {
  clear_error();
  HG_REQUIRE(n_evaluated, "hg_ransac_adaptive: NULL n_evaluated");
  HG_REQUIRE(confidence > 0.0 && confidence < 1.0, "hg_ransac_adaptive: confidence must be in (0, 1)");
  if (int st = check_batched(corr, ld, off, n_pairs, n_hyp_max, thresh, tune, best_H, best_count,
                             best_hyp, inlier_mask, ws, ws_bytes))
    return st;
  const size_t need = hg_ransac_adaptive_ws_bytes(n_pairs, n_hyp_max);
  if (ws_bytes < need)
    return fail(HG_EWORKSPACE, "hg_ransac_adaptive: workspace of %zu bytes needed, %zu given",
                need, ws_bytes);
  hg_ransac_tuning t = tune ? *tune : lookup_tune(n_pairs, n_hyp_max);
  t.hyps_per_block = kRound;   // a work item is one round
  // without an explicit shape: at most 4 workgroups per CU (more rounds in
  // flight at once means more speculative rounds past the stopping points)
  if (!tune) t.blocks_per_cu = std::min(t.blocks_per_cu, 4);
  RansacArgs a = make_args(corr, ld, off, 0, n_pairs, n_hyp_max, kRound, thresh, seed, best_H,
                           best_count, best_hyp, inlier_mask, nullptr);
  char *x = static_cast<char *>(ws) + batched_ws_bytes(n_pairs);
  a.pst = reinterpret_cast<PairState *>(x);
  x += align256(sizeof(PairState) * static_cast<size_t>(n_pairs));
  a.rkey = reinterpret_cast<unsigned long long *>(x);
  x += align256(8ull * n_pairs * a.n_hb);
  if (stagger_rounds(n_pairs, a.n_hb)) a.iorder = reinterpret_cast<int32_t *>(x);
  a.n_eval = n_evaluated;
  a.one_minus_conf = 1.0 - confidence;
  return launch_batched(a, t, ws, as_stream(stream));
}

extern "C" int hg_ransac_batched_graph_create(const float *corr, int64_t ld, const int64_t *off,
                                              int32_t n_pairs, int32_t n_hyp, float thresh,
                                              uint64_t seed, const hg_ransac_tuning *tune,
                                              float *best_H, int32_t *best_count,
                                              int32_t *best_hyp, uint8_t *inlier_mask,
                                              int32_t *hyp_counts, void *ws, size_t ws_bytes,
                                              void *stream, hg_graph **out) {
  clear_error();
  HG_REQUIRE(out, "hg_ransac_batched_graph_create: NULL out");
  *out = nullptr;
  if (int st = check_batched(corr, ld, off, n_pairs, n_hyp, thresh, tune, best_H, best_count,
                             best_hyp, inlier_mask, ws, ws_bytes))
    return st;
  const hg_ransac_tuning t = tune ? *tune : lookup_tune(n_pairs, n_hyp);
  RansacArgs a = make_args(corr, ld, off, 0, n_pairs, n_hyp, t.hyps_per_block, thresh, seed,
                           best_H, best_count, best_hyp, inlier_mask, hyp_counts);
  return capture_graph(stream, [&](hipStream_t cap) { return launch_batched(a, t, ws, cap); },
                       out);
}

extern "C" int hg_graph_launch(hg_graph *g, void *stream) {
  clear_error();
  HG_REQUIRE(g && g->exec, "hg_graph_launch: NULL graph");
  HG_HIP(hipGraphLaunch(g->exec, as_stream(stream)));
  return HG_OK;
}

extern "C" void hg_graph_destroy(hg_graph *g) {
  if (!g) return;
  if (g->exec) (void)hipGraphExecDestroy(g->exec);
  if (g->graph) (void)hipGraphDestroy(g->graph);
  delete g;
}
