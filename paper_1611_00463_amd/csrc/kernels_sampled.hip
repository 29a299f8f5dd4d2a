// Step 6 of Section IV in one pass: the handler merges all P runs a partition
// received at once (F = the power of two reaching P), with tile boundaries
// chosen the way the paper chooses its splitters, by regular sampling.
//
// Every run (block i's slice for partition k) offers as samples the elements
// at its positions 0, m, 2m, ...; or, where the local sort writes block
// samples (64-bit keys: the group fix-up writes its blocks in position
// order, so writing the keys at block positions that are multiples of m to a
// side array costs little there, while a radix pass would scatter them), its
// first element and the elements at the block positions after it that are
// multiples of m, read from that side array: about 1/m of the keys instead of
// a strided read that touches every cache line.  Either way consecutive
// samples of a run, and the last one and the run's end, are at most m apart.  The samples of block i, taken run by run, are a sorted
// sequence, and the sample runs of partition k have the structure of the
// main problem at about 1/m of its size: they are merged per partition by
// the multi-pass handler (exact merge-path tiles), which orders them by
// (key, run, position), the order of the stable merge.
//
// Tile j of partition k spans from the sample of sorted rank j*q to the one of
// rank (j+1)*q (the first tile starts at the partition's start, the last ends
// at its end).  A boundary b that is a sample cuts run i at the number of its
// elements that precede b in that order: elements <= b's key for runs before
// b's own run, < b's key for runs after it, and b's position in its own run.
// If samples 0 .. s-1 of run i (at run positions p_0 = 0 < p_1 < ...) precede
// b and sample s does not, that count lies in (p_{s-1}, p_s] (p_s = the run's
// length past its last sample; 0 when s = 0).  Between two boundaries with q
// samples between them a run gains at most p_{s'} - p_{s-1} <= m (s' - s + 1)
// elements, so a tile holds at most m q + P m elements whatever the keys
// (heavy duplicates included): q is chosen so that this is the merge tile's
// capacity.  No selection rounds are needed: one binary search per run and
// boundary.
#include "lbsort_internal.hpp"

namespace lbs {

// Per instance: sample counts of every run, the sample problem's block starts,
// cut matrix and range table (the same layout as the main problem's), and per
// partition the sorted samples' start and the number of merge tiles.
// Instance b's samples start at floor(start of its first block / m) +
// b (P^2 + 1), which is at least the number of samples of all instances
// before it (the block starts are the validated segment table; all zero for a
// malformed one, whose blocks are empty).
__global__ __launch_bounds__(256) void k_samp_meta(Plan p, SampPlan sp) {
  __shared__ u32 s_ns[64 * 64];
  __shared__ u64 s_tot[64];
  __shared__ u64 s_G[65];
  const u32 b = blockIdx.x, tid = threadIdx.x;
  const u32 P = p.P, m = sp.m;
  const u64* c = p.cuts + (u64)b * P * (P + 1);
  for (u32 x = tid; x < P * P; x += 256) {
    // run (i, k) = block positions [c0, c0 + C): its first element and the
    // multiples of m after it
    const u32 i = x / P, k = x % P;
    const u64 c0 = c[(u64)i * (P + 1) + k], C = c[(u64)i * (P + 1) + k + 1] - c0;
    if (p.bsamp)
      s_ns[x] = C ? (u32)(1 + (c0 + C - 1) / m - c0 / m) : 0u;
    else
      s_ns[x] = (u32)((C + m - 1) / m);  // run positions 0, m, 2m, ...
  }
  __syncthreads();
  u64* sc = sp.scuts + (u64)b * P * (P + 1);
  for (u32 i = tid; i < P; i += 256) {
    u64 run = 0;
    for (u32 k = 0; k < P; ++k) {
      sc[(u64)i * (P + 1) + k] = run;
      run += s_ns[i * P + k];
    }
    sc[(u64)i * (P + 1) + P] = run;
    s_tot[i] = run;
  }
  for (u32 k = tid; k < P; k += 256) {
    u64 col = 0;
    for (u32 i = 0; i < P; ++i) col += s_ns[i * P + k];
    s_G[k + 1] = col;
  }
  __syncthreads();
  const u64 PP1 = 2 * (u64)P * P + 1;
  const u64 base = p.blk_start[(u64)b * P] / m + (u64)b * PP1;
  if (tid == 0) {
    sp.sseg[b] = base;
    u64 at = base;
    for (u32 i = 0; i < P; ++i) {
      sp.sbs[(u64)b * P + i] = at;
      at += s_tot[i];
    }
    if (b + 1 == p.B) {
      sp.sseg[p.B] = p.blk_start[(u64)p.B * P] / m + (u64)p.B * PP1;
      sp.sbs[(u64)p.B * P] = sp.sseg[p.B];
    }
    s_G[0] = 0;
    for (u32 k = 0; k < P; ++k) s_G[k + 1] += s_G[k];
  }
  __syncthreads();
  u64* Db = sp.sDm + (u64)b * (P + 1) * P;
  for (u32 k = tid; k < P; k += 256) {
    u64 acc = s_G[k];
    for (u32 i = 0; i < P; ++i) {
      Db[(u64)i * P + k] = acc;
      acc += s_ns[i * P + k];
    }
    Db[(u64)P * P + k] = s_G[k + 1];
    const u64 ns = s_G[k + 1] - s_G[k];
    sp.gsbase[(u64)b * P + k] = base + s_G[k];
    sp.ntile[(u64)b * P + k] = (u32)((ns + sp.q - 1) / sp.q);
  }
}

// One thread per sample slot u of the sample problem: its block (the last
// sample block starting at or before u), its run (the last sample cut at or
// before u inside the block) and its index j in the run; it copies the run's
// element j*m and, as its value, that element's position in the sorted
// blocks (32-bit).  Slots in the gaps between instances do nothing.
template <typename K>
__global__ __launch_bounds__(256) void k_samp_gather(Plan p, SampPlan sp, const K* __restrict__ sorted,
                                                     K* __restrict__ skeys, u32* __restrict__ svals) {
  __shared__ u32 s_rng[2];
  const u64 u0 = (u64)blockIdx.x * 256, u = u0 + threadIdx.x;
  const u32 P = p.P, NB = p.B * P;
  const u64 total = sp.sseg[p.B];
  if (u0 >= total) return;  // the whole workgroup
  const u32 bi = wg_find_seg(sp.sbs, NB, u, u0, min(u0 + 255, total - 1), s_rng);
  if (u >= total) return;
  const u64 off = u - sp.sbs[bi];
  const u64* sc = sp.scuts + (u64)bi * (P + 1);
  if (u < sp.sbs[bi] || off >= sc[P]) return;  // a gap between instances
  u32 k = 0;
  {
    u32 lo = 0, hi = P;
    while (hi - lo > 1) {
      const u32 mid = (lo + hi) >> 1;
      if (sc[mid] <= off) lo = mid; else hi = mid;
    }
    k = lo;
  }
  // sample j of the run: its first element (j = 0), else the j-th block
  // position after it that is a multiple of m, whose key the local sort
  // wrote to the block samples
  const u64 j = off - sc[k];
  const u64 bs = p.blk_start[bi], c0 = p.cuts[(u64)bi * (P + 1) + k];
  if (!p.bsamp) {
    // no block samples: the run's elements at run positions 0, m, 2m, ...
    const u64 at = bs + c0 + j * sp.m;
    skeys[u] = sorted[at];
    svals[u] = (u32)at;
  } else if (j == 0) {
    skeys[u] = sorted[bs + c0];
    svals[u] = (u32)(bs + c0);
  } else {
    const u64 xm = c0 / sp.m + j;  // block position / m
    skeys[u] = ((const K*)p.bsamp)[bs / sp.m + bi + xm];
    svals[u] = (u32)(bs + xm * sp.m);
  }
}

// Prefix of the merge tiles over the partitions of all instances (one
// workgroup).
__global__ __launch_bounds__(1024) void k_samp_tiles(Plan p, SampPlan sp) {
  __shared__ u64 s_w[16];
  const u32 tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const u32 NG = p.B * p.P;
  u64 carry = 0;
  for (u32 base = 0; base < NG; base += 1024) {
    const u32 g = base + tid;
    const u64 nt = g < NG ? sp.ntile[g] : 0;
    u64 x = nt;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
      const u64 y = __shfl_up(x, o);
      if (lane >= (u32)o) x += y;
    }
    if (lane == 63) s_w[w] = x;
    __syncthreads();
    if (w == 0) {
      u64 t = lane < 16 ? s_w[lane] : 0;
#pragma unroll
      for (int o = 1; o < 16; o <<= 1) {
        const u64 y = __shfl_up(t, o);
        if (lane >= (u32)o) t += y;
      }
      if (lane < 16) s_w[lane] = t;
    }
    __syncthreads();
    if (g < NG) p.mtile[g] = (u32)(carry + (w ? s_w[w - 1] : 0) + x - nt);
    carry += s_w[15];
    __syncthreads();
  }
  if (tid == 0) p.mtile[NG] = (u32)carry;
}

// One wave per merge tile: the cuts of its starting boundary in every run
// (lane i: run i), written as the tile's run starts and as the previous
// tile's run ends; the last tile of a partition also ends every run.
template <typename K, bool UPPER>
__device__ inline u64 count_before(const K* a, u64 lo, u64 hi, K x) {
  return bsearch_count<K, UPPER>(a, lo, hi, x) - lo;
}

template <typename K>
__global__ __launch_bounds__(256) void k_samp_bounds(Plan p, SampPlan sp, const K* __restrict__ sorted,
                                                     const K* __restrict__ skeys, const u32* __restrict__ svals) {
  const u32 t = (blockIdx.x * 256 + threadIdx.x) >> 6;
  const u32 lane = threadIdx.x & 63;
  const u32 P = p.P, F = p.F, NG = p.B * P;
  if (t >= p.mtile[NG]) return;
  const u32 g = wave_find_seg(p.mtile, NG, t);  // the partition holding tile t (empty ones skipped)
  const u32 j = t - p.mtile[g], nt = p.mtile[g + 1] - p.mtile[g];
  const u32 b = g / P, k = g % P;
  u64 base = 0, len = 0;
  if (lane < P) {
    const u64 bi = (u64)b * P + lane;
    const u64* c = p.cuts + bi * (P + 1);
    base = p.blk_start[bi] + c[k];
    len = c[k + 1] - c[k];
  }
  u64 cut = 0;
  if (j > 0) {
    const u64 si = sp.gsbase[g] + (u64)j * sp.q;
    const K v = skeys[si];
    const u64 gp = svals[si];
    // the boundary's own run: the block whose start is the last one <= gp
    const u64* bs = p.blk_start + (u64)b * P;
    u32 r = 0;
    {
      u32 lo = 0, hi = P;
      while (hi - lo > 1) {
        const u32 mid = (lo + hi) >> 1;
        if (bs[mid] <= gp) lo = mid; else hi = mid;
      }
      r = lo;
    }
    if (lane < P) {
      if (lane == r) cut = gp - base;
      else if (lane < r) cut = count_before<K, true>(sorted, base, base + len, v);
      else cut = count_before<K, false>(sorted, base, base + len, v);
      if (cut > len) cut = len;  // only a malformed sample could get here
    }
  }
  u64 tot = cut;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) tot += __shfl_xor(tot, o);
  if (lane < F) {
    const u64 at = lane < P ? base + cut : 0;
    p.rec_start[(u64)t * F + lane] = at;
    if (j > 0) p.rec_end[(u64)(t - 1) * F + lane] = at;
    if (j + 1 == nt) p.rec_end[(u64)t * F + lane] = lane < P ? base + len : 0;
  }
  if (lane == 0) {
    const u64* Db = p.Dm + (u64)b * (P + 1) * P;
    p.rec_out[t] = p.seg[b] + Db[k] + tot;
    p.rec_n[t] = p.TM;
  }
}

template <typename K, bool HASV>
void launch_merge_sampled(const Plan& p, u32 NG, u64 max_tiles, const K* src, const u32* srcv, K* dst, u32* dstv,
                          hipStream_t s);
template <typename K, bool HASV>
void launch_merge_level(const Plan& p, u32 level, const K* src, const u32* srcv, K* dst, u32* dstv, hipStream_t s);

// The whole one-pass handler: sample metadata, the samples, their merge per
// partition (ps: the sample problem's plan, L_s passes), tile bounds, and the
// merge of the data.  sorted: the local sort's output; the result goes to dst.
template <typename K, bool HASV>
void launch_handler_sampled(const Plan& p, const Plan& ps, const SampPlan& sp, u64 max_tiles, const K* sorted,
                            const u32* sortedv, K* dst, u32* dstv, hipStream_t s) {
  const u32 NG = p.B * p.P;
  { const int pe_ = prof_begin(s); hipLaunchKernelGGL(k_samp_meta, dim3(p.B), dim3(256), 0, s, p, sp); prof_end(pe_, "samp_meta", s); }
  { const int pe_ = prof_begin(s); hipLaunchKernelGGL(k_samp_gather<K>, dim3((u32)((ps.total_n + 255) / 256)), dim3(256), 0, s, p, sp,
                     sorted, (K*)sp.skeys[0], sp.svals[0]); prof_end(pe_, "samp_gather", s); }
  // the samples' merge per partition: the multi-pass handler on the sample problem
  for (u32 l = 0; l < ps.L; ++l)
    launch_merge_level<K, true>(ps, l, (const K*)sp.skeys[l & 1], sp.svals[l & 1], (K*)sp.skeys[(l + 1) & 1],
                                sp.svals[(l + 1) & 1], s);
  const K* sk = (const K*)sp.skeys[ps.L & 1];
  const u32* sv = sp.svals[ps.L & 1];
  { const int pe_ = prof_begin(s); hipLaunchKernelGGL(k_samp_tiles, dim3(1), dim3(1024), 0, s, p, sp); prof_end(pe_, "samp_tiles", s); }
  { const int pe_ = prof_begin(s); hipLaunchKernelGGL(k_samp_bounds<K>, dim3((u32)((max_tiles + 3) / 4)), dim3(256), 0, s, p, sp, sorted,
                     sk, sv); prof_end(pe_, "samp_bounds", s); }
  launch_merge_sampled<K, HASV>(p, NG, max_tiles, sorted, sortedv, dst, dstv, s);
}

template void launch_handler_sampled<u32, false>(const Plan&, const Plan&, const SampPlan&, u64, const u32*, const u32*,
                                                 u32*, u32*, hipStream_t);
template void launch_handler_sampled<u32, true>(const Plan&, const Plan&, const SampPlan&, u64, const u32*, const u32*,
                                                u32*, u32*, hipStream_t);
template void launch_handler_sampled<u64, false>(const Plan&, const Plan&, const SampPlan&, u64, const u64*, const u32*,
                                                 u64*, u32*, hipStream_t);
template void launch_handler_sampled<u64, true>(const Plan&, const Plan&, const SampPlan&, u64, const u64*, const u32*,
                                                u64*, u32*, hipStream_t);

}  // namespace lbs
