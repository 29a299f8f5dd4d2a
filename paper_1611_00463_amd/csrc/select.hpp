// Wave-wide multi-sequence selection shared by the merge partition and the
// splitter selection.
#pragma once
#include "lbsort_internal.hpp"

namespace lbs {

// ----------------------------------------------------------------- selection
// Split of the first `a` elements of the stable merge of F sorted runs (order:
// key, then run, then position).  Lane l works on run l % F.  Each round every
// run with a non-empty window [lo, hi) offers QPR pivots at evenly spaced
// positions; for every pivot every lane counts, inside its own run's window,
// the elements that precede the pivot (binary search, M searches per lane).
// The clamped counts sum to less than `a` exactly when the pivot is among the
// first `a` elements, and each decided pivot moves lo or hi of every run.
// Every round strictly shrinks every non-empty window, so the loop ends with
// lo = hi = the split.
template <typename K, int F, int M>
__device__ inline u64 wave_select(const K* __restrict__ src, u64 roff, u64 lo, u64 hi, u64 a, u32* counters) {
  constexpr int NPIV = 64 * M / F;
  constexpr int QPR = NPIV / F;
  static_assert(QPR >= 1, "every run needs a pivot per round");
  const u32 lane = threadIdx.x & 63;
  const u32 r = lane % F;
  for (int round = 0; round < 96; ++round) {
    // widest window of the wave: every lane runs the same number of steps
    u64 wmax = hi - lo, wsum = hi - lo, lsum = lo;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
      const u64 y = __shfl_xor(wmax, o);
      wmax = y > wmax ? y : wmax;
    }
    if (wmax == 0) return lo;
#pragma unroll
    for (int o = 1; o < F; o <<= 1) {
      wsum += __shfl_xor(wsum, o);
      lsum += __shfl_xor(lsum, o);
    }
    // The first round puts the pivots around the proportional guess
    // lo + (a - sum lo) W / sum W; later rounds spread them evenly.
    u64 pos[M], base[M];
    K px[M];
    bool pvalid[M];
    u32 own[M];
#pragma unroll
    for (int m = 0; m < M; ++m) {
      const u32 s = lane + 64 * m;
      const u32 piv = s / F;
      own[m] = piv % F;
      const u32 qi = piv / F;
      const u64 lo_o = __shfl(lo, (int)own[m]);
      const u64 hi_o = __shfl(hi, (int)own[m]);
      const u64 off_o = __shfl(roff, (int)own[m]);
      const u64 W = hi_o - lo_o;
      pvalid[m] = W > 0;
      u64 at = lo_o + (W * (qi + 1)) / (QPR + 1);
      if (round == 0 && wsum > 0) {
        // only a starting point (any position in the window is correct), so
        // floating point is enough: 0 <= a - sum lo <= sum W keeps it in range
        const u64 guess = lo_o + (u64)((double)(a - lsum) * (double)W / (double)wsum);
        const u64 d = W / 64 > 1 ? W / 64 : 1;
        const int k = (int)qi - QPR / 2;  // -QPR/2 .. QPR/2-1
        const u64 mag = d << (2 * (k < 0 ? -k - 1 : k));
        u64 want = k < 0 ? (guess > mag ? guess - mag : 0) : guess + mag - (k == 0 ? d : 0);
        at = want < lo_o ? lo_o : (want >= hi_o ? (hi_o > 0 ? hi_o - 1 : 0) : want);
      }
      pos[m] = at;
      px[m] = pvalid[m] ? src[off_o + pos[m]] : (K)0;
      base[m] = lo;
    }
    // M interleaved searches over this lane's run window [lo, hi), power-of-two
    // steps: base ends at lo + #elements of the window that precede the pivot.
    u64 step = 1;
    while (step * 2 <= wmax) step *= 2;
    for (; step > 0; step >>= 1) {
      K v[M];
#pragma unroll
      for (int m = 0; m < M; ++m) {
        const bool ok = base[m] + step <= hi;
        v[m] = ok ? src[roff + base[m] + step - 1] : (K)0;
      }
#pragma unroll
      for (int m = 0; m < M; ++m) {
        const bool ok = base[m] + step <= hi;
        const bool before = (r < own[m]) ? (v[m] <= px[m]) : (v[m] < px[m]);
        if (ok && before) base[m] += step;
      }
    }
    u64 nlo = lo, nhi = hi;
#pragma unroll
    for (int m = 0; m < M; ++m) {
      const u64 c = (own[m] == r) ? pos[m] : base[m];
      u64 tot = c;
#pragma unroll
      for (int o = 1; o < F; o <<= 1) tot += __shfl_xor(tot, o);
      if (pvalid[m]) {
        if (tot < a) {
          const u64 cand = (own[m] == r) ? pos[m] + 1 : c;
          nlo = cand > nlo ? cand : nlo;
        } else {
          nhi = c < nhi ? c : nhi;
        }
      }
    }
#pragma unroll
    for (int o = F; o < 64; o <<= 1) {
      const u64 ol = __shfl_xor(nlo, o), oh = __shfl_xor(nhi, o);
      nlo = ol > nlo ? ol : nlo;
      nhi = oh < nhi ? oh : nhi;
    }
    lo = nlo;
    hi = nhi;
  }
  if (lane == 0) set_error(counters, E_SELECT);
  return lo;
}

}  // namespace lbs
