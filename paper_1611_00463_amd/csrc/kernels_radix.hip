// Step 1 of Section IV on the GPU: every block (virtual processor) is sorted
// on its own by a stable least-significant-digit radix sort (the paper names
// radix sort in Section II; its own step 1 uses quicksort, which is not
// stable).  One pass per 8-bit digit.  Each pass is a single kernel in the
// "onesweep" style (Adinets and Merrill, 2022): per-block digit counts of all
// passes are taken up front, and a tile finds where its keys go from the
// running counts of the earlier tiles of the same block, published through a
// decoupled look-back chain with ordered tile ids.
//
// Ranking inside a tile uses wave-wide ballots on the 8 digit bits (a
// match-any), mbcnt for the rank among equal digits, and per-wave counters in
// LDS; keys are then staged in LDS in digit order so that the global writes
// are runs of consecutive addresses.
#include "lbsort_internal.hpp"

namespace lbs {

constexpr u32 SPIN_LIMIT = 1u << 22;

// ----------------------------------------------------------------- scans
template <int NT>
__device__ inline u64 block_exclusive_scan(u64 v, u64* s_w, u64& total) {
  const u32 lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  constexpr int NWV = NT / 64;
  u64 x = v;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    u64 y = __shfl_up(x, o);
    if (lane >= (u32)o) x += y;
  }
  if (lane == 63) s_w[w] = x;
  __syncthreads();
  if (w == 0) {
    u64 t = lane < NWV ? s_w[lane] : 0;
#pragma unroll
    for (int o = 1; o < NWV; o <<= 1) {
      u64 y = __shfl_up(t, o);
      if (lane >= (u32)o) t += y;
    }
    if (lane < NWV) s_w[lane] = t;
  }
  __syncthreads();
  u64 wprefix = w ? s_w[w - 1] : 0;
  total = s_w[NWV - 1];
  __syncthreads();
  return wprefix + x - v;
}

// ----------------------------------------------------------------- plan
// One workgroup: block starts, radix tile prefix, list of blocks small enough
// to be sorted whole in LDS, and sample offsets, for every block of every
// instance.  A malformed segment table latches E_SEG and every block is
// treated as empty so that no later kernel reads out of range.
__global__ __launch_bounds__(1024) void k_plan(Plan p) {
  __shared__ u64 s_w[16];
  __shared__ u32 s_bad;
  __shared__ u32 s_qmin[NQ];
  __shared__ u64 s_qb1[NQ], s_qb2[NQ];
  const u32 tid = threadIdx.x;
  if (tid == 0) s_bad = (p.seg[0] != 0 || p.seg[p.B] != p.total_n) ? 1u : 0u;
  __syncthreads();
  for (u32 b = tid; b < p.B; b += 1024) {
    if (p.seg[b + 1] < p.seg[b]) s_bad = 1u;
    // generated values are 32-bit input positions
    else if (p.vidx && p.seg[b + 1] - p.seg[b] > (1ull << 32)) set_error(p.counters, E_RANGE);
  }
  __syncthreads();
  const bool bad = s_bad != 0;
  if (bad && tid == 0) set_error(p.counters, E_SEG);
  // BPT consecutive blocks per thread and round, their loads issued together
  constexpr u32 BPT = 8;
  u64 carry_t = 0, carry_s = 0, carry_m = 0, carry_l = 0;
  for (u32 base = 0; base < p.NB; base += 1024 * BPT) {
    const u32 i0 = base + tid * BPT;
    u64 tiles[BPT], smp[BPT];
    bool small[BPT];
    u64 st = 0, ss = 0, sl = 0, sm = 0;
#pragma unroll
    for (u32 j = 0; j < BPT; ++j) {
      const u32 idx = i0 + j;
      u64 n = 0, bs = 0;
      if (idx < p.NB) {
        const u32 b = idx / p.P, i = idx % p.P;
        if (!bad) {
          bs = block_begin(p.seg, b, i, p.P);
          n = block_begin(p.seg, b, i + 1, p.P) - bs;
        }
        if (n >= (1ull << 32)) {
          set_error(p.counters, E_RANGE);
          n = 0;
        }
        p.blk_start[idx] = bs;
      }
      // with a filter, only the listed large blocks are planned (small blocks
      // and sample offsets are unaffected by it)
      const bool keep = (p.only == nullptr || (idx < p.NB && p.only[idx] != 0)) &&
                        (p.skip == nullptr || (idx < p.NB && p.skip[idx] == 0));
      tiles[j] = (keep && n > (u64)SMALL_TILE) ? (n + p.rtile - 1) / p.rtile : 0;
      smp[j] = n < (u64)p.s ? n : (u64)p.s;
      small[j] = p.only == nullptr && n > 0 && n <= (u64)SMALL_TILE;
      st += tiles[j];
      sl += tiles[j] ? 1 : 0;
      ss += smp[j];
      sm += small[j] ? 1 : 0;
    }
    u64 tot_t, tot_l, tot_s, tot_m;
    u64 et = carry_t + block_exclusive_scan<1024>(st, s_w, tot_t);
    u64 el = carry_l + block_exclusive_scan<1024>(sl, s_w, tot_l);
    u64 es = carry_s + block_exclusive_scan<1024>(ss, s_w, tot_s);
    u64 em = carry_m + block_exclusive_scan<1024>(sm, s_w, tot_m);
#pragma unroll
    for (u32 j = 0; j < BPT; ++j) {
      const u32 idx = i0 + j;
      if (idx < p.NB) {
        p.tstart[idx] = (u32)et;
        p.samp_start[idx] = es;
      }
      if (tiles[j]) p.large_list[el++] = idx;
      if (small[j]) p.small_list[em++] = idx;
      et += tiles[j];
      es += smp[j];
    }
    carry_t += tot_t;
    carry_l += tot_l;
    carry_s += tot_s;
    carry_m += tot_m;
  }
  if (tid == 0) p.tstart[p.NB] = (u32)carry_t;
  __syncthreads();
  // Tile queues: large block j goes to queue j % nq.  Per queue: block count,
  // fewest tiles (rmin), prefix of the tiles beyond the interleaved head, and
  // the queue's first slot in the look-back status array.  All queues in one
  // scan: the large blocks in queue-major order (queue x's blocks jx = 0, 1,
  // ... at k = qoff(x) + jx), each queue's prefix being the scan minus its
  // value at the queue's first block.
  const u32 nl = (u32)carry_l;
  const u32 nq = p.nq;
  const u32 qa = nl / nq, qr = nl % nq;  // queue x holds qa + (x < qr) blocks
  auto qoff = [&](u32 x) { return x * qa + (x < qr ? x : qr); };
  if (tid < NQ) {
    s_qmin[tid] = 0xFFFFFFFFu;
    s_qb1[tid] = s_qb2[tid] = 0;
  }
  __syncthreads();
  for (u32 j = tid; j < nl; j += 1024) {
    const u32 blk = p.large_list[j];
    atomicMin(&s_qmin[j % nq], p.tstart[blk + 1] - p.tstart[blk]);
  }
  __syncthreads();
  u64 carry_r = 0, carry_q = 0;
  for (u32 base = 0; base < nl; base += 1024 * BPT) {
    const u32 k0 = base + tid * BPT;
    u32 tl[BPT], jj[BPT], xx[BPT];
    u64 sr = 0, sq = 0;
#pragma unroll
    for (u32 i = 0; i < BPT; ++i) {
      const u32 k = k0 + i;
      tl[i] = 0;
      xx[i] = 0;
      jj[i] = 0;
      if (k < nl) {
        // queue and index of the k-th block in queue-major order
        const u32 head = qr * (qa + 1);
        const u32 x = k < head ? k / (qa + 1) : qr + (k - head) / qa;
        const u32 jx = k - qoff(x);
        xx[i] = x;
        jj[i] = x + nq * jx;
        const u32 blk = p.large_list[jj[i]];
        tl[i] = p.tstart[blk + 1] - p.tstart[blk];
      }
      sr += tl[i] ? tl[i] - s_qmin[xx[i]] : 0;
      sq += tl[i];
    }
    u64 tot, totq;
    u64 er = carry_r + block_exclusive_scan<1024>(sr, s_w, tot);
    u64 eq = carry_q + block_exclusive_scan<1024>(sq, s_w, totq);
#pragma unroll
    for (u32 i = 0; i < BPT; ++i) {
      const u32 k = k0 + i;
      if (k < nl) {
        if (k == qoff(xx[i])) {  // the queue's first block: its bases
          s_qb1[xx[i]] = er;
          s_qb2[xx[i]] = eq;
        }
        p.rem_prefix[jj[i]] = (u32)er;  // made queue-relative below
      }
      er += tl[i] ? tl[i] - s_qmin[xx[i]] : 0;
      eq += tl[i];
    }
    carry_r += tot;
    carry_q += totq;
  }
  __syncthreads();
  for (u32 j = tid; j < nl; j += 1024) p.rem_prefix[j] -= (u32)s_qb1[j % nq];
  if (tid < nq) {
    const u32 x = tid, nbx = qa + (x < qr ? 1u : 0u);
    const u64 qbase = nbx ? s_qb2[x] : carry_q;
    const u64 qend = x + 1 < nq && qa + (x + 1 < qr ? 1u : 0u) ? s_qb2[x + 1] : carry_q;
    p.counters[C_QPARAM + 4 * x + 0] = nbx;
    p.counters[C_QPARAM + 4 * x + 1] = nbx ? s_qmin[x] : 0;
    p.counters[C_QPARAM + 4 * x + 2] = (u32)qbase;
    p.counters[C_QPARAM + 4 * x + 3] = (u32)(nbx ? qend - qbase : 0);
  }
  if (tid == 0) {
    p.samp_start[p.NB] = carry_s;
    p.blk_start[p.NB] = bad ? 0 : p.seg[p.B];
    p.counters[C_NSMALL] = (u32)carry_m;
    p.counters[C_NLARGE] = nl;
  }
}

// Status slot g of the radix passes (queue x owns slots [qbase_x, qbase_x +
// tiles_x), ticket order): its block, tile and key range.
__global__ __launch_bounds__(256) void k_tile_desc(Plan p) {
  const u32 g = blockIdx.x * 256 + threadIdx.x;
  for (u32 x = 0; x < p.nq; ++x) {
    const u32 qbase = p.counters[C_QPARAM + 4 * x + 2], qtiles = p.counters[C_QPARAM + 4 * x + 3];
    if (g < qbase || g - qbase >= qtiles) continue;
    const TileQueue Q{x, p.nq, p.counters[C_QPARAM + 4 * x], p.counters[C_QPARAM + 4 * x + 1], p.rem_prefix};
    u32 jx, lt;
    Q.locate(g - qbase, jx, lt);
    const u32 blk = p.large_list[x + p.nq * jx];
    TileDesc d;
    d.bstart = p.blk_start[blk];
    d.tbase = d.bstart + (u64)lt * p.rtile;
    const u64 rem = p.blk_start[blk + 1] - d.tbase;
    d.blk = blk;
    d.lt = lt;
    d.jx = jx;
    d.tile_n = rem < (u64)p.rtile ? (u32)rem : p.rtile;
    d.tail = Q.nb * Q.rmin + Q.rem(jx) - Q.rmin;
    d.pad = 0;
    p.tdesc[g] = d;
    return;
  }
}

// Several fills in one launch (FillSet: up to FILL_MAX ranges).
__global__ void k_fill_set(FillSet f) {
  const u64 stride = (u64)gridDim.x * blockDim.x;
  for (int r = 0; r < f.count; ++r)
    for (u64 i = (u64)blockIdx.x * blockDim.x + threadIdx.x; i < f.n[r]; i += stride) f.a[r][i] = f.v[r];
}

// ----------------------------------------------------------------- histogram
// Digit counts of all passes for the tiles of large blocks, accumulated per
// block.  A workgroup covers `tpw` consecutive tiles (block-contiguous
// numbering; at most HIST_TILES, fewer when there are few tiles so that the
// grid still covers the chip) and flushes its LDS counts to the block's global
// counts when the block changes, so global atomics are few.  Equal keys inside a wave are
// first merged (the wave's remembered hot key, then a few leader rounds) so
// that heavy duplicates do not serialise on one LDS counter.
constexpr u32 HIST_TILES = 16;
constexpr int LOOKBACK = 4;  // predecessors read per look-back round

// Digit positions DLO..D-1 are counted (the others stay zero).
template <typename K, int DLO>
__global__ __launch_bounds__(SORT_NT) void k_hist(Plan p, const K* __restrict__ src, u32 tpw) {
  constexpr int D = KeyT<K>::BITS / RADIX_BITS;
  __shared__ u32 h[D * RADIX];
  __shared__ u32 s_blk;
  const u32 tid = threadIdx.x, lane = tid & 63;
  const u32 total = p.tstart[p.NB];
  const u32 t_begin = blockIdx.x * tpw;
  if (t_begin >= total) return;
  const u32 t_end = t_begin + tpw < total ? t_begin + tpw : total;
  for (int i = tid; i < D * RADIX; i += SORT_NT) h[i] = 0;
  if (tid == 0) s_blk = find_seg(p.tstart, p.NB, t_begin);
  __syncthreads();
  u32 blk = s_blk;
  K hot = 0;
  bool have_hot = false;
  // Presorted blocks: every pair of neighbours inside the block is compared;
  // a pair out of non-decreasing order clears bit 0 of the block's flag, one
  // out of non-increasing order bit 1 (one atomic per wave and block).
  bool up_ok = true, down_ok = true;
  auto flush_order = [&](u32 b) {
    if (p.presorted == nullptr) return;
    const u32 clear = (__ballot(!up_ok) ? 1u : 0u) | (__ballot(!down_ok) ? 2u : 0u);
    if (clear && lane == 0) atomicAnd(&p.presorted[b], ~clear);
    up_ok = down_ok = true;
  };
  for (u32 t = t_begin; t < t_end; ++t) {
    if (t >= p.tstart[blk + 1]) {
      // next block: flush the counts of this one
      flush_order(blk);
      __syncthreads();
      u32* gh = p.hist + (u64)blk * D * RADIX;
      for (int i = tid; i < D * RADIX; i += SORT_NT) {
        if (h[i]) atomicAdd(&gh[i], h[i]);
        h[i] = 0;
      }
      while (t >= p.tstart[blk + 1]) ++blk;
      __syncthreads();
    }
    const u64 tbase = p.blk_start[blk] + (u64)(t - p.tstart[blk]) * p.rtile;
    const u64 rem = p.blk_start[blk + 1] - tbase;
    const u32 tile_n = rem < (u64)p.rtile ? (u32)rem : p.rtile;
    // the tile's keys are read HB at a time, all loads in flight together
    // (a load and its use in one step made every key wait on memory alone)
    constexpr int HB = 8;
    static_assert((RTILE_SMALL / SORT_NT) % HB == 0 && (RTILE_LARGE / SORT_NT) % HB == 0 &&
                  (RTILE_HUGE / SORT_NT) % HB == 0, "whole load batches");
    const int per_thread = (int)(p.rtile / SORT_NT);
    for (int j0 = 0; j0 < per_thread; j0 += HB) {
    // order checks only while some lane of the wave has not yet seen a pair
    // out of each order (random keys stop checking after a few keys)
    const bool chk = p.presorted != nullptr && __ballot(up_ok || down_ok) != 0;
    K kb[HB], kn[HB];
#pragma unroll
    for (int u = 0; u < HB; ++u) {
      const u32 idx = (j0 + u) * SORT_NT + tid;
      kb[u] = src[tbase + (idx < tile_n ? idx : 0)];  // clamped: tile_n >= 1
      // the last lane of a wave also needs the key after its own (the next
      // wave's first, or the next tile's): loaded with the others
      kn[u] = (chk && lane == 63 && (u64)idx + 1 < rem) ? src[tbase + idx + 1] : (K)0;
    }
#pragma unroll
    for (int u = 0; u < HB; ++u) {
      const u32 idx = (j0 + u) * SORT_NT + tid;
      const bool valid = idx < tile_n;
      const K key = valid ? key_in<K>(kb[u], p.kx_top, p.kx_fm) : (K)0;
      if (chk) {
        // the key at idx + 1: the next lane's, or for the last lane of the
        // wave a load (the next wave's first key, or the next tile's)
        K nxt = __shfl_down(key, 1);
        const bool pair = (u64)idx + 1 < rem;
        if (lane == 63) nxt = key_in<K>(kn[u], p.kx_top, p.kx_fm);
        if (valid && pair) {
          up_ok = up_ok && key <= nxt;
          down_ok = down_ok && key >= nxt;
        }
      }
      bool done = !valid;
      if (have_hot) {
        // the wave's hot key (a value seen in many lanes before) first
        const u64 hm = __ballot(valid && key == hot);
        if (__popcll(hm) >= 2) {
          if (lane == (u32)(__ffsll((unsigned long long)hm) - 1)) {
            const u32 c = (u32)__popcll(hm);
#pragma unroll
            for (int q = DLO; q < D; ++q) atomicAdd(&h[q * RADIX + (u32)((hot >> (q * RADIX_BITS)) & (RADIX - 1))], c);
          }
          done = done || key == hot;
        }
      }
      // leader rounds on the first key of each load batch only: they find
      // the hot key of duplicate-heavy data, and on spread keys they cost
      // more than the collisions they would save
      for (int r = 0; r < (u == 0 ? 3 : 0); ++r) {
        const u64 act = __ballot(!done);
        if (act == 0) break;
        const int leader = __ffsll((unsigned long long)act) - 1;
        const K lk = lane_value(key, leader);
        const bool same = !done && key == lk;
        const u64 sm = __ballot(same);
        if (__popcll(sm) < 2) break;  // no duplicate of the leader: leave all to the bulk path
        if (__popcll(sm) >= 8) {
          hot = lk;
          have_hot = true;
        }
        if (lane == (u32)leader) {
          const u32 c = (u32)__popcll(sm);
#pragma unroll
          for (int q = DLO; q < D; ++q) atomicAdd(&h[q * RADIX + (u32)((lk >> (q * RADIX_BITS)) & (RADIX - 1))], c);
        }
        done = done || same;
      }
      // the rest, digit by digit.  Counting every digit (the fallback plan of
      // 64-bit keys, 32-bit keys), a digit the remaining lanes share (a run
      // of equal high bytes, as in clustered or small keys) is counted once;
      // the top digits of the fix-up path count lane by lane (cheaper on
      // spread keys, the common case there).
      const u64 rest = __ballot(!done);
      if (DLO > 0) {
        if (!done) {
#pragma unroll
          for (int q = DLO; q < D; ++q) atomicAdd(&h[q * RADIX + (u32)((key >> (q * RADIX_BITS)) & (RADIX - 1))], 1u);
        }
      } else if (rest) {
        const int first = __ffsll((unsigned long long)rest) - 1;
#pragma unroll
        for (int q = DLO; q < D; ++q) {
          const u32 d = (u32)((key >> (q * RADIX_BITS)) & (RADIX - 1));
          const u32 d0 = lane_value(d, first);
          if (__ballot(!done && d != d0) == 0) {
            if (lane == (u32)first) atomicAdd(&h[q * RADIX + d0], (u32)__popcll(rest));
          } else if (!done) {
            atomicAdd(&h[q * RADIX + d], 1u);
          }
        }
      }
    }
    }
  }
  flush_order(blk);
  __syncthreads();
  u32* gh = p.hist + (u64)blk * D * RADIX;
  for (int i = tid; i < D * RADIX; i += SORT_NT)
    if (h[i]) atomicAdd(&gh[i], h[i]);
}

// Presorted large blocks (step 1 needs no radix pass for them; TimSort's runs
// are the same idea): a workgroup takes PRESORTED_TPW consecutive radix tiles
// of the full plan and writes their keys (mapped to the unsigned order) and
// values to the local sort's output.  A non-decreasing block is copied; a non-increasing one is reversed
// run by run: the key at block position x whose run of equal keys is [a, b)
// goes to n - b + (x - a), which keeps equal keys in input order (stable).
// Runs are found from the neighbours in the common case of distinct keys, by
// binary search in the block otherwise.  Tiles of other blocks leave at once.
constexpr u32 PRESORTED_TPW = 1;  // radix tiles per workgroup of k_presorted

template <typename K, bool HASV>
__global__ __launch_bounds__(256) void k_presorted(Plan p, const K* __restrict__ src, const u32* __restrict__ srcv,
                                                   K* __restrict__ dst, u32* __restrict__ dstv) {
  constexpr int U = 8;  // elements per thread per round, their loads issued together
  __shared__ u32 s_blk;
  const u32 tid = threadIdx.x;
  const u32 ntiles = p.tstart[p.NB];
  const u32 t0 = blockIdx.x * PRESORTED_TPW;
  if (t0 >= ntiles) return;
  // one workgroup per tile: the block by a wave-wide search (a batch has
  // tens of thousands of blocks)
  if (tid < 64) {
    const u32 b = wave_find_seg(p.tstart, p.NB, t0);
    if (tid == 0) s_blk = b;
  }
  __syncthreads();
  u32 blk = s_blk;
  const u32 t1 = t0 + PRESORTED_TPW < ntiles ? t0 + PRESORTED_TPW : ntiles;
  for (u32 t = t0; t < t1; ++t) {
    while (t >= p.tstart[blk + 1]) ++blk;  // consecutive tiles: the same block or a later one
    const u32 f = p.presorted[blk];
    if (f == 0) continue;
    const u64 bs = p.blk_start[blk], be = p.blk_start[blk + 1];
    const u64 tbase = bs + (u64)(t - p.tstart[blk]) * p.rtile;
    const u32 tile_n = be - tbase < (u64)p.rtile ? (u32)(be - tbase) : p.rtile;
    const u64 vgen = bs - p.seg[blk / p.P];  // generated values: input position inside the instance
    const u64 n = be - bs;
    for (u32 i0 = 0; i0 < tile_n; i0 += 256 * U) {
      K kk[U];
      u32 vv[U];
      // every load issued (past the tile a lane reads the tile's first
      // element and writes nothing), so that each store waits for its own
      // element's loads only
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const u32 i = i0 + (u32)u * 256 + tid;
        const u64 xc = tbase + (i < tile_n ? i : 0u);
        kk[u] = src[xc];
        vv[u] = 0;
        if (HASV) vv[u] = srcv != nullptr ? srcv[xc] : (u32)(vgen + (xc - bs));
      }
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const u32 i = i0 + (u32)u * 256 + tid;
        if (i >= tile_n) continue;
        const u64 x = tbase + i;
        const K k = key_in<K>(kk[u], p.kx_top, p.kx_fm);
        u64 o = x;
        if ((f & 1u) == 0) {
          // non-increasing: the run of k is [a, b) (block-relative)
          const u64 xr = x - bs;
          const bool eq_prev = xr > 0 && key_in<K>(src[x - 1], p.kx_top, p.kx_fm) == k;
          const bool eq_next = xr + 1 < n && key_in<K>(src[x + 1], p.kx_top, p.kx_fm) == k;
          u64 a = xr, b = xr + 1;
          if (eq_prev || eq_next) {
            // keys above k come first, then the run of k, then keys below it
            u64 lo = 0, hi = n;
            while (lo < hi) {
              const u64 mid = lo + ((hi - lo) >> 1);
              if (key_in<K>(src[bs + mid], p.kx_top, p.kx_fm) > k) lo = mid + 1; else hi = mid;
            }
            a = lo;
            hi = n;
            while (lo < hi) {
              const u64 mid = lo + ((hi - lo) >> 1);
              if (key_in<K>(src[bs + mid], p.kx_top, p.kx_fm) >= k) lo = mid + 1; else hi = mid;
            }
            b = lo;
          }
          o = bs + (n - b) + (xr - a);
        }
        dst[o] = k;
        if (HASV) dstv[o] = vv[u];
        block_sample<K>(p, blk, bs, o, k);
      }
    }
  }
}

// Exclusive scan of the 256 counts of every (block, pass): digit start offsets.
__global__ __launch_bounds__(256) void k_scan_hist(Plan p) {
  const u32 gw = (blockIdx.x * blockDim.x + threadIdx.x) >> 6;
  const u32 lane = threadIdx.x & 63;
  if (gw >= p.NB * p.D) return;
  const u32 blk = gw / p.D;
  if (p.tstart[blk + 1] == p.tstart[blk]) return;
  u32* h = p.hist + (u64)gw * RADIX;
  const u32 a0 = h[lane * 4 + 0], a1 = h[lane * 4 + 1], a2 = h[lane * 4 + 2], a3 = h[lane * 4 + 3];
  const u32 s = a0 + a1 + a2 + a3;
  if (p.run_slot) {
    // two or more non-empty buckets: the pass over this digit reorders the block
    const u32 nzl = (a0 != 0) + (a1 != 0) + (a2 != 0) + (a3 != 0);
    const bool varies = __popcll(__ballot(nzl != 0)) >= 2 || __ballot(nzl >= 2) != 0;
    if (varies && lane == 0) atomicOr(&p.counters[p.run_slot], 1u << (gw % p.D));
  }
  u32 x = s;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    u32 y = __shfl_up(x, o);
    if (lane >= (u32)o) x += y;
  }
  const u32 ex = x - s;
  h[lane * 4 + 0] = ex;
  h[lane * 4 + 1] = ex + a0;
  h[lane * 4 + 2] = ex + a0 + a1;
  h[lane * 4 + 3] = ex + a0 + a1 + a2;
}

// ----------------------------------------------------------------- ranking
// Items are laid out wave-major: item j of lane l of wave w is tile position
// w*64*ITEMS + j*64 + l, so processing j in order and lanes in order inside a
// wave keeps the ranking stable.  wc: this wave's 256 digit counters.
template <typename K, int ITEMS, typename C>
__device__ inline void rank_items(const K (&keys)[ITEMS], u32 wbase, u32 tile_n, u32 shift, C* wc,
                                  u32 (&rank)[ITEMS], u32 (&dig)[ITEMS], int nj = ITEMS) {
  const u32 lane = threadIdx.x & 63;
#pragma unroll
  for (int j = 0; j < ITEMS; ++j) {
    if (j >= nj) break;  // items past a wave-uniform count hold no keys
    const bool valid = wbase + j * 64 + lane < tile_n;
    const u32 d = (u32)(keys[j] >> shift) & (RADIX - 1);
    // Peers: lanes whose digit equals this lane's.  For every digit bit the
    // lane's bit is spread to a full-word mask t (signed one-bit extract);
    // t ^ ballot marks the lanes whose bit differs, and each 32-bit half of
    // the peer set keeps the lanes marked by no bit: plo &= ~(t ^ ballot), one
    // three-input bit operation (truth table 0x90) per half and bit.  The
    // empty asm keeps t opaque, so that the ballot tests t itself instead of
    // a second shift of the digit.
    const u64 vm = __ballot(valid);
    u32 plo = (u32)vm, phi = (u32)(vm >> 32);
#pragma unroll
    for (int b = 0; b < RADIX_BITS; ++b) {
      u32 t = (u32)__builtin_amdgcn_sbfe((int)d, b, 1);
      asm("" : "+v"(t));
      const u64 bb = __ballot(t != 0u);
      plo = __builtin_amdgcn_bitop3_b32(plo, t, (u32)bb, 0x90);
      phi = __builtin_amdgcn_bitop3_b32(phi, t, (u32)(bb >> 32), 0x90);
    }
    const u64 m = ((u64)phi << 32) | plo;
    const u32 below = count_below(m);
    u32 base = 0;
    if (valid) base = wc[d];
    if (valid && below == 0) wc[d] = (C)(base + (u32)__popcll(m));
    rank[j] = base + below;
    dig[j] = d;
  }
}

// ----------------------------------------------------------------- one pass
// Persistent workgroups: workgroup w serves queue w % nq first (the hardware
// hands workgroups to the XCDs round-robin), then helps the other queues.
// A tile waits only for tiles of its own queue with smaller tickets, which
// running workgroups hold, so the waits always end.
// REDO: a pass of the fallback plan (blocks the group fix-up flagged); it is
// a separate instantiation so that profiles tell the two apart, and it
// leaves at once when the plan holds no block.  With p.run_slot set, a pass
// over a digit that is the same for all keys of every block does not run,
// and the passes that do run choose their buffers: the first reads the
// input (src0), the last writes p.pass_out.
template <typename K, bool HASV, int NT, int ITEMS, int MINW, bool REDO>
__global__ __launch_bounds__(NT, MINW) void k_onesweep(Plan p, const K* __restrict__ src0,
                                                 const u32* __restrict__ srcv0, K* __restrict__ dst0,
                                                 u32* __restrict__ dstv0, u32 pass) {
  constexpr int NWV = NT / 64, WI = 64 * ITEMS;
  constexpr u32 TILE = NT * ITEMS;  // the launch passes this kernel only calls whose p.rtile == TILE
  static_assert(TILE == RTILE_SMALL || TILE == RTILE_LARGE || (TILE == RTILE_HUGE && sizeof(K) == 4),
                "radix tiles of RTILE_SMALL or RTILE_LARGE keys, RTILE_HUGE for 32-bit keys");
  static_assert(NT >= RADIX, "one thread per digit");
  // LDS: 16-bit per-wave digit counters (they end up holding the tile-local
  // start of each wave's run of a digit), 32-bit block-relative write bases,
  // and the tile staged in digit order.  With 8 items per thread keys and
  // values are staged together; with 16 (SPLITV) the values are loaded and
  // staged after the keys have gone out, in the same buffer, so that neither
  // the registers nor the LDS hold both (two 8192-key workgroups per compute
  // unit stay within 80 KB each).  One struct, small fields first, so that
  // they sit at addresses the LDS instructions' immediate offsets reach.
  constexpr bool SPLITV = HASV && ITEMS > 8;
  struct Smem {
    u32 ticket;    // current ticket
    TileDesc td;   // its tile
    u64 scan[NWV];
    u32 gbase[RADIX];
    uint16_t wc[NWV][RADIX];
    K stage[TILE];
    u32 vstage[HASV && !SPLITV ? TILE : 1];
  };
  __shared__ Smem sm;
  auto& s_scan = sm.scan;
  auto& s_gbase = sm.gbase;
  auto& s_wc = sm.wc;
  auto& s_stage = sm.stage;
  auto& s_vstage = sm.vstage;
  // The workgroup's current ticket and its tile.  Thread 0 fetches the next
  // ticket and tile while the current one is processed, so that per tile only
  // the key loads wait on memory.  A tile still waits only for tiles with
  // smaller tickets: the smallest unfinished ticket is always one a running
  // workgroup is processing (any ticket held ahead belongs to a workgroup
  // whose current tile is smaller), so the waits always end.
  auto& s_ticket = sm.ticket;
  auto& s_td = sm.td;
  const u32 tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const u32 shift = pass * RADIX_BITS;
  const u32 epoch = pass + 1 + p.epoch_base;
  const u32 nq = p.nq;
  const K* src = src0;
  const u32* srcv = srcv0;
  K* dst = dst0;
  u32* dstv = dstv0;
  u64 kx_top = p.kx_top, kx_fm = p.kx_fm;  // applied to keys read from the input only
  if (REDO && p.counters[C_NLARGE] == 0) return;
  // the last pass writes the local sort's output: its block samples too
  bool emit = p.bsamp != nullptr && pass + 1 == p.D;
  if (p.run_slot) {
    u32 run = p.counters[p.run_slot] & p.run_mask;
    if (run == 0) run = 1u << (31 - __clz(p.run_mask));  // at least one pass writes pass_out
    if (((run >> pass) & 1u) == 0) return;
    const u32 a = (u32)__popc(run & ((1u << pass) - 1u)), e = (u32)__popc(run);
    emit = p.bsamp != nullptr && a + 1 == e;
    // the k-th pass that runs writes pass_out when e - 1 - k is even
    const bool to_out = ((e - 1u - a) & 1u) == 0;
    dst = (K*)(to_out ? p.pass_out : p.pass_tmp);
    dstv = to_out ? p.pass_outv : p.pass_tmpv;
    if (a > 0) {
      src = (const K*)(to_out ? p.pass_tmp : p.pass_out);
      srcv = to_out ? p.pass_tmpv : p.pass_outv;
      kx_top = kx_fm = 0;
    }
  }
  for (u32 qi = 0; qi < nq; ++qi) {
    const u32 x = (blockIdx.x + qi) % nq;
    const TileQueue Q{x, nq, p.counters[C_QPARAM + 4 * x], p.counters[C_QPARAM + 4 * x + 1], p.rem_prefix};
    const u32 qbase = p.counters[C_QPARAM + 4 * x + 2];
    const u32 qtiles = p.counters[C_QPARAM + 4 * x + 3];
    u32* const ticket = &p.counters[C_TICKET + nq * pass + x];
    __syncthreads();
    if (tid == 0) {
      const u32 t0 = atomicAdd(ticket, 1u);
      s_ticket = t0;
      if (t0 < qtiles) s_td = p.tdesc[qbase + t0];
    }
    while (true) {
      for (int i = tid; i < NWV * RADIX; i += NT) (&s_wc[0][0])[i] = 0;
      __syncthreads();
      // the tile's numbers are the same in every lane: keep them in scalars
      const u32 t = __builtin_amdgcn_readfirstlane(s_ticket);
      if (t >= qtiles) break;
      const u32 blk = __builtin_amdgcn_readfirstlane(s_td.blk), lt = __builtin_amdgcn_readfirstlane(s_td.lt);
      const u32 jx = __builtin_amdgcn_readfirstlane(s_td.jx), tile_n = __builtin_amdgcn_readfirstlane(s_td.tile_n);
      const u32 tail = __builtin_amdgcn_readfirstlane(s_td.tail);
      // status slot of tile u of this block, without memory accesses (the
      // look-back requests its window at once)
      auto slot_of = [&](u32 u) { return u < Q.rmin ? u * Q.nb + jx : tail + u; };
      const u64 bstart = uniform_u64(s_td.bstart), tbase = uniform_u64(s_td.tbase);
      u32 nt = 0;
      if (tid == 0) nt = atomicAdd(ticket, 1u);
      u32 hv = 0;
      const u32* const hrow = p.hist + ((u64)blk * p.D + pass) * RADIX;
      if (tid < RADIX) hv = hrow[tid];
      const u32 wbase = w * WI;

      // (SPLITV: the values are loaded after the keys have gone out)
      K keys[ITEMS];
      u32 vals[HASV && !SPLITV ? ITEMS : 1];
      if (!HASV || SPLITV || srcv != nullptr) {
        // The keys' loads first, then the values'.  Every load is issued (a
        // lane past the tile reads the tile's first element, which it never
        // uses: its ranking, staging and writes are masked), so that the
        // compiler knows how many loads follow each one and item j waits for
        // keys[j] alone; a load skipped by a branch would make the ranking
        // wait for all of them.
#pragma unroll
        for (int j = 0; j < ITEMS; ++j) {
          const u32 idx = wbase + j * 64 + lane;
          keys[j] = src[tbase + (idx < tile_n ? idx : 0u)];
        }
        if (HASV && !SPLITV) {
#pragma unroll
          for (int j = 0; j < ITEMS; ++j) {
            const u32 idx = wbase + j * 64 + lane;
            vals[j] = srcv[tbase + (idx < tile_n ? idx : 0u)];
          }
        }
      } else {
        // no value array: the values are the keys' input positions inside
        // their instance (a separate loop, so that the key loads stay in
        // flight together)
        const u64 vgen = tbase - p.seg[blk / p.P];
#pragma unroll
        for (int j = 0; j < ITEMS; ++j) {
          const u32 idx = wbase + j * 64 + lane;
          keys[j] = src[tbase + (idx < tile_n ? idx : 0u)];
          if (HASV && !SPLITV) vals[j] = (u32)(vgen + idx);
        }
      }
      if ((kx_top | kx_fm) != 0) {
#pragma unroll
        for (int j = 0; j < ITEMS; ++j) keys[j] = key_in<K>(keys[j], kx_top, kx_fm);
      }
      u32 rank[ITEMS];
      {
        u32 dig[ITEMS];
        rank_items<K, ITEMS, uint16_t>(keys, wbase, tile_n, shift, s_wc[w], rank, dig);
      }
      // The next tile's record, read by wave 0 into wave-uniform scalars (a
      // struct here would be placed in LDS, per-lane copies cost registers).
      const u32 ntu = __builtin_amdgcn_readfirstlane(nt);
      u64 nd_bstart = 0, nd_tbase = 0;
      u32 nd_blk = 0, nd_lt = 0, nd_jx = 0, nd_n = 0, nd_tail = 0;
      if (__builtin_amdgcn_readfirstlane(w) == 0 && ntu < qtiles) {
        const TileDesc* q = p.tdesc + qbase + ntu;
        nd_bstart = q->bstart;
        nd_tbase = q->tbase;
        nd_blk = q->blk;
        nd_lt = q->lt;
        nd_jx = q->jx;
        nd_n = q->tile_n;
        nd_tail = q->tail;
      }
      __syncthreads();

      // Per-digit tile count.
      const u32 d = tid < RADIX ? tid : 0;
      u32 tot = 0;
#pragma unroll
      for (int v = 0; v < NWV; ++v) tot += s_wc[v][d];
      if (tid >= RADIX) tot = 0;
      // Decoupled look-back over the earlier tiles of this block, digit = tid.
      // The tile's aggregate is published and the first LOOKBACK predecessors
      // are requested at once; the tile-local scan and the staging of the keys
      // run while those loads are in flight, and the walk over them (in
      // registers) follows.  A look-back that ends inside the window costs
      // one memory round trip, mostly hidden.
      u64* st = p.status + (u64)(qbase + t) * RADIX + d;
      const bool lookback = tid < RADIX && lt > 0;
      u32 plt = lt - 1;  // next predecessor to add
      u64 v[LOOKBACK];
      if (tid < RADIX) st_release_agent(st, st_pack(epoch, lt == 0 ? ST_INC : ST_AGG, tot));
      if (lookback) {
#pragma unroll
        for (int i = 0; i < LOOKBACK; ++i)
          v[i] = (u32)i <= plt ? ld_acquire_agent(p.status + (u64)(qbase + slot_of(plt - i)) * RADIX + d) : 0;
      }
      u64 ttot;
      const u32 lstart = (u32)block_exclusive_scan<NT>(tot, s_scan, ttot);
      if (tid < RADIX) {
        // per-wave counts become each wave's tile-local start of the digit
        u32 run = lstart;
#pragma unroll
        for (int wv = 0; wv < NWV; ++wv) {
          const u32 c = s_wc[wv][tid];
          s_wc[wv][tid] = (uint16_t)run;
          run += c;
        }
      }
      __syncthreads();
#pragma unroll
      for (int j = 0; j < ITEMS; ++j) {
        rank[j] += s_wc[w][(u32)(keys[j] >> shift) & (RADIX - 1)];  // rank[] now holds the staged position
        if (wbase + j * 64 + lane < tile_n) {
          s_stage[rank[j]] = keys[j];
          if (HASV && !SPLITV) s_vstage[rank[j]] = vals[j];
        }
      }
      u64 excl = 0;
      if (lookback) {
        u32 spins = 0;
        while (true) {
          bool done = false;
          u32 used = 0;
#pragma unroll
          for (int i = 0; i < LOOKBACK; ++i) {
            if (done || used != (u32)i || (u32)i > plt || (u32)(v[i] >> 56) != epoch) continue;
            excl += v[i] & ST_VALMASK;
            used = i + 1;
            done = ((v[i] >> 54) & 3u) == ST_INC || plt == (u32)i;
          }
          if (done) break;
          plt -= used;
          if (used == 0) {  // the next predecessor has not published yet
            if (++spins > SPIN_LIMIT) {
              set_error(p.counters, E_SPIN);
              break;
            }
            __builtin_amdgcn_s_sleep(1);
          }
#pragma unroll
          for (int i = 0; i < LOOKBACK; ++i)
            v[i] = (u32)i <= plt ? ld_acquire_agent(p.status + (u64)(qbase + slot_of(plt - i)) * RADIX + d) : 0;
        }
        st_release_agent(st, st_pack(epoch, ST_INC, excl + tot));
      }
      // Every thread read this tile's s_ticket and s_td before the barrier
      // after the ranking; the next tile's record has arrived by now.
      if (tid == 0) {
        s_ticket = ntu;
        s_td.bstart = nd_bstart;
        s_td.tbase = nd_tbase;
        s_td.blk = nd_blk;
        s_td.lt = nd_lt;
        s_td.jx = nd_jx;
        s_td.tile_n = nd_n;
        s_td.tail = nd_tail;
      }
      if (tid < RADIX) s_gbase[tid] = (u32)(hv + excl - lstart);
      __syncthreads();
      K* const dblk = dst + bstart;
      u32* const vblk = HASV ? dstv + bstart : nullptr;
      // Write-out: staged position i = j * NT + tid goes to its digit's base
      // + i.  The LDS reads of a chunk of CH items first, then its stores, so
      // that the LDS latency is paid once per chunk rather than once per item.
      constexpr int CH = ITEMS < 8 ? ITEMS : 8;
      u32 oo[SPLITV ? ITEMS : 1];
#pragma unroll
      for (int c = 0; c < ITEMS; c += CH) {
        K ok[CH];
        u32 oc[CH];
        u32 ov[HASV && !SPLITV ? CH : 1];
#pragma unroll
        for (int j = 0; j < CH; ++j) {
          const u32 i = (u32)(c + j) * NT + tid;
          ok[j] = i < tile_n ? s_stage[i] : (K)0;
          if (HASV && !SPLITV) ov[j] = i < tile_n ? s_vstage[i] : 0u;
        }
#pragma unroll
        for (int j = 0; j < CH; ++j) {
          oc[j] = s_gbase[(u32)(ok[j] >> shift) & (RADIX - 1)] + (u32)(c + j) * NT + tid;
          if (SPLITV) oo[c + j] = oc[j];
        }
#pragma unroll
        for (int j = 0; j < CH; ++j)
          if ((u32)(c + j) * NT + tid < tile_n) {
            dblk[oc[j]] = ok[j];
            if (HASV && !SPLITV) vblk[oc[j]] = ov[j];
            if (emit) block_sample<K>(p, blk, bstart, bstart + oc[j], ok[j]);
          }
      }
      if (SPLITV) {
        // the values, through the same buffer once every key has been read
        // from it; staged position and destination are the keys'
        u32* const s_vs = reinterpret_cast<u32*>(&s_stage[0]);
        u32 vv[ITEMS];
        if (srcv != nullptr) {
#pragma unroll
          for (int j = 0; j < ITEMS; ++j) {
            const u32 idx = wbase + j * 64 + lane;
            vv[j] = idx < tile_n ? srcv[tbase + idx] : 0u;
          }
        } else {
          const u64 vgen = tbase - p.seg[blk / p.P];
#pragma unroll
          for (int j = 0; j < ITEMS; ++j) vv[j] = (u32)(vgen + wbase + j * 64 + lane);
        }
        __syncthreads();
#pragma unroll
        for (int j = 0; j < ITEMS; ++j)
          if (wbase + j * 64 + lane < tile_n) s_vs[rank[j]] = vv[j];
        __syncthreads();
#pragma unroll
        for (int j = 0; j < ITEMS; ++j) {
          const u32 i = (u32)j * NT + tid;
          if (i < tile_n) vblk[oo[j]] = s_vs[i];
        }
      }
    }
  }
}

// ----------------------------------------------------------------- group fix-up
// Second phase of the local sort of 64-bit keys.  The large blocks arrive
// stably sorted by key >> p.gshift (radix passes over the three highest
// digits, the four highest for doubles); a group is a run of keys with equal
// top bits, and each group must
// end up sorted by the whole key, stably.  One workgroup per tile of a large
// block, with a window of GF_HALO keys on either side in LDS:
//  * a group of at most GF_HALO keys lies inside the window of every tile
//    that holds one of its keys; each key's place is the group start plus
//    the number of group members before it in (key, position) order;
//  * a larger group keeps its order, which is right when all its keys are
//    equal (heavy duplicates); a key of it that differs from its predecessor
//    flags the block for k_group_fix_mid.

// The fix-ups work on parts of GF1_SPAN keys of a radix tile (rtile /
// GF1_SPAN parts per tile), so that their LDS window is small enough for
// several workgroups per compute unit.
constexpr u32 GF1_SPAN = RTILE_SMALL;
constexpr int GF1_NT = 512;
constexpr u32 GF1_WIN = GF1_SPAN + 2 * GF_HALO;

template <bool HASV>
__global__ __launch_bounds__(GF1_NT) void k_group_fix(Plan p, const u64* __restrict__ src,
                                                    const u32* __restrict__ srcv, u64* __restrict__ dst,
                                                    u32* __restrict__ dstv) {
  constexpr u32 NW = GF1_WIN / 64 + 2;  // head-bit words, with room for the block's end
  __shared__ u64 s_k[GF1_WIN];
  __shared__ u64 s_hb[NW];  // bit w: window position w starts a group
  __shared__ u32 s_blk;
  const u32 tid = threadIdx.x, lane = tid & 63;
  const u32 split = p.rtile / GF1_SPAN;
  const u32 t = blockIdx.x / split, part = blockIdx.x % split;  // radix tile and its part
  if (t >= p.tstart[p.NB]) return;
  if (tid == 0) s_blk = find_seg(p.tstart, p.NB, t);
  for (u32 i = tid; i < NW; i += GF1_NT) s_hb[i] = 0;
  __syncthreads();
  const u32 blk = s_blk;
  const u64 bs = p.blk_start[blk], be = p.blk_start[blk + 1];
  const u64 ts = bs + (u64)(t - p.tstart[blk]) * p.rtile + (u64)part * GF1_SPAN;
  if (ts >= be) return;  // the last tile of a block may not reach this part
  const u64 te = be - ts < (u64)GF1_SPAN ? be : ts + GF1_SPAN;
  const u64 ws = ts - bs > GF_HALO ? ts - GF_HALO : bs;
  const u64 we = be - te > GF_HALO ? te + GF_HALO : be;
  const u32 wn = (u32)(we - ws);
  const bool wfirst = ws == bs, wlast = we == be;
  const u32 gsh = p.gshift;  // groups: equal key >> gsh
  // all loads issued at once: the window's keys (into LDS) and this thread's
  // values of the tile (kept in registers until the write)
  constexpr int KL = (GF1_WIN + GF1_NT - 1) / GF1_NT, VL = GF1_SPAN / GF1_NT;
  const u32 o0 = (u32)(ts - ws), o1 = (u32)(te - ws);
  u32 v[HASV ? VL : 1];
  if (HASV) {
#pragma unroll
    for (int k = 0; k < VL; ++k) {
      const u32 w = o0 + (u32)k * GF1_NT + tid;
      v[k] = w < o1 ? srcv[ws + w] : 0u;
    }
  }
  {
    u64 kk[KL];
#pragma unroll
    for (int k = 0; k < KL; ++k) {
      const u32 i = (u32)k * GF1_NT + tid;
      kk[k] = i < wn ? src[ws + i] : 0;
    }
#pragma unroll
    for (int k = 0; k < KL; ++k) {
      const u32 i = (u32)k * GF1_NT + tid;
      if (i < wn) s_k[i] = kk[k];
    }
  }
  __syncthreads();
  // Position w starts a group when it is the block's first key or its top
  // bits differ from those at w - 1; the window's first position inside a
  // block is no start (a group reaching past it counts as large), and the
  // block's end counts as one.  One ballot per 64 positions.
  for (u32 base = 0; base < wn + 1; base += GF1_NT) {
    const u32 w = base + tid;
    bool h = false;
    if (w < wn) h = w == 0 ? wfirst : (s_k[w] >> gsh) != (s_k[w - 1] >> gsh);
    else if (w == wn) h = wlast;
    const u64 m = __ballot(h);
    if (lane == 0 && w < wn + 64) s_hb[w >> 6] = m;
  }
  __syncthreads();
  bool bad = false;
#pragma unroll
  for (int k = 0; k < VL; ++k) {
    const u32 w = o0 + (u32)k * GF1_NT + tid;
    if (w >= o1) break;
    const u64 key = s_k[w];
    // group bounds within 64 positions: the last start at or before w and the
    // first start after it (a group of at most GF_HALO keys has both there)
    const u32 wi = w >> 6, b = w & 63;
    const u64 upto = ((u64)2 << b) - 1;  // bits 0..b
    u32 gs = 0xFFFFFFFFu, ge = 0xFFFFFFFFu;
    u64 m = s_hb[wi] & upto;
    if (m) gs = wi * 64 + 63 - (u32)__clzll((long long)m);
    else if (wi > 0 && (m = s_hb[wi - 1]) != 0) gs = (wi - 1) * 64 + 63 - (u32)__clzll((long long)m);
    m = s_hb[wi] & ~upto;
    if (m) ge = wi * 64 + (u32)__ffsll((long long)m) - 1;
    else if ((m = s_hb[wi + 1]) != 0) ge = (wi + 1) * 64 + (u32)__ffsll((long long)m) - 1;
    u32 o = w;
    if (gs != 0xFFFFFFFFu && ge != 0xFFFFFFFFu && ge - gs <= GF_HALO) {
      u32 r = 0;
      for (u32 j = gs; j < ge; ++j) {
        const u64 kj = s_k[j];
        r += (kj < key || (kj == key && j < w)) ? 1u : 0u;
      }
      o = gs + r;
    } else if (gs != w && s_k[w - 1] != key) {
      bad = true;  // a large group with different keys (w >= 1: w = 0 only at a block start)
    }
    dst[ws + o] = key;
    if (HASV) dstv[ws + o] = v[k];
    block_sample<u64>(p, blk, bs, ws + o, key);
  }
  // one store per wave that found a mixed large group
  if (__ballot(bad) != 0 && lane == 0) {
    p.gflags[blk] = 1u;
    p.counters[C_ANYFLAG] = 1u;
  }
}

template <bool HASV>
void launch_group_fix(const Plan& p, const u64* src, const u32* srcv, u64* dst, u32* dstv, hipStream_t s) {
  if (p.max_tiles == 0) return;
  const int pe_ = prof_begin(s);
  hipLaunchKernelGGL(k_group_fix<HASV>, dim3(p.max_tiles * (p.rtile / GF1_SPAN)), dim3(GF1_NT), 0, s, p, src, srcv, dst, dstv);
  prof_end(pe_, "group_fix", s);
}
template void launch_group_fix<false>(const Plan&, const u64*, const u32*, u64*, u32*, hipStream_t);
template void launch_group_fix<true>(const Plan&, const u64*, const u32*, u64*, u32*, hipStream_t);

// ----------------------------------------------------------------- mid-size group fix-up
// The fix-up again, for the blocks k_group_fix flagged (a group of more than
// GF_HALO keys with different keys).  One workgroup per tile of such a block.
// It holds the tile and GF_HALO keys on either side in LDS, and marks group
// starts over a wider window of GF_MID keys on either side (from the top bits
// alone), so that every group of at most GF_MID keys that touches the tile is
// seen whole:
//  * a group of at most GF_HALO keys: each key's place is the group start
//    plus the number of group members before it in (key, position) order;
//  * a group of GF_HALO+1 .. GF_MID keys is listed (by the tile holding its
//    first key) for k_group_mid, which sorts it in LDS and writes it;
//  * a larger group keeps its order, which is right when all its keys are
//    equal (heavy duplicates); a key of it that differs from its predecessor
//    flags the block again (gflags2), which is then sorted over all eight
//    digits.
constexpr u32 GF_XWIN = GF1_SPAN + 2 * GF_MID;
constexpr u32 GF_MIDPART = GF1_SPAN / (GF_HALO + 1) + 1;  // listed groups starting in one part, at most

template <bool HASV>
__global__ __launch_bounds__(GF1_NT) void k_group_fix_mid(Plan p, const u64* __restrict__ src,
                                                    const u32* __restrict__ srcv, u64* __restrict__ dst,
                                                    u32* __restrict__ dstv) {
  constexpr u32 NW = GF_XWIN / 64 + 2;      // head-bit words, with room for the block's end
  constexpr u32 XH = GF_MID - GF_HALO;      // outer halo: top bits only
  __shared__ u64 s_k[GF1_WIN + 1];           // keys of the tile and the inner halo (+ one spill slot)
  __shared__ u32 s_xt[2][XH];               // top bits of the outer halo, left and right
  __shared__ u64 s_hb[NW];                  // bit x: window position x starts a group
  __shared__ u32 s_last[NW];                // last group start in words <= w (or none)
  __shared__ u32 s_first[NW];               // first group start in words >= w (or none)
  __shared__ u64 s_mid[GF_MIDPART];  // mid-size groups starting in the tile
  __shared__ u32 s_nmid, s_mbase, s_empty;
  __shared__ u32 s_blk;
  const u32 tid = threadIdx.x, lane = tid & 63;
  const u32 split = p.rtile / GF1_SPAN;
  const u32 t = blockIdx.x / split, part = blockIdx.x % split;  // radix tile and its part
  if (p.counters[C_ANYFLAG] == 0 || t >= p.tstart[p.NB]) return;  // no block flagged
  if (tid == 0) {
    s_blk = find_seg(p.tstart, p.NB, t);
    s_nmid = 0;
    s_empty = 0;
  }
  for (u32 i = tid; i < NW; i += GF1_NT) s_hb[i] = 0;
  __syncthreads();
  const u32 blk = s_blk;
  if (p.gflags[blk] == 0) return;  // the first fix-up finished this block
  const u64 bs = p.blk_start[blk], be = p.blk_start[blk + 1];
  const u64 ts = bs + (u64)(t - p.tstart[blk]) * p.rtile + (u64)part * GF1_SPAN;
  if (ts >= be) return;  // the last tile of a block may not reach this part
  const u64 te = be - ts < (u64)GF1_SPAN ? be : ts + GF1_SPAN;
  // inner window [ws, we) in LDS
  const u64 ws = ts - bs > GF_HALO ? ts - GF_HALO : bs;
  const u64 we = be - te > GF_HALO ? te + GF_HALO : be;
  const u32 wn = (u32)(we - ws);
  const u32 gsh = p.gshift;  // groups: equal key >> gsh (32 or 40)
  // all loads issued at once: the inner window's keys (into LDS) and this
  // thread's values of the tile (kept in registers until the write)
  constexpr int KL = (GF1_WIN + GF1_NT - 1) / GF1_NT, VL = GF1_SPAN / GF1_NT;
  const u32 o0 = (u32)(ts - ws), o1 = (u32)(te - ws);
  u32 v[HASV ? VL : 1];
  if (HASV) {
#pragma unroll
    for (int k = 0; k < VL; ++k) {
      const u32 w = o0 + (u32)k * GF1_NT + tid;
      v[k] = w < o1 ? srcv[ws + w] : 0u;
    }
  }
  {
    u64 kk[KL];
#pragma unroll
    for (int k = 0; k < KL; ++k) {
      const u32 i = (u32)k * GF1_NT + tid;
      kk[k] = src[ws + (i < wn ? i : wn - 1)];  // clamped, not predicated: all loads in flight together
    }
    // positions past wn take clamped copies, which nothing reads; those past
    // the array go to its spill slot (no predicated store, so that no load
    // is moved behind the wait of the others)
#pragma unroll
    for (int k = 0; k < KL; ++k) {
      const u32 i = (u32)k * GF1_NT + tid;
      s_k[i < GF1_WIN ? i : GF1_WIN] = kk[k];
    }
  }
  __syncthreads();
  // The outer window [xs, xe) reaches GF_MID keys past the tile on a side
  // only where the group at that edge of the tile runs to the edge of the
  // inner window (equal top bits there, since the keys are sorted by them);
  // elsewhere every group touching the tile starts and ends inside.
  const bool need_l = ws > bs && (s_k[0] >> gsh) == (s_k[o0] >> gsh);
  const bool need_r = we < be && (s_k[wn - 1] >> gsh) == (s_k[o1 - 1] >> gsh);
  const u64 xs = need_l ? (ts - bs > GF_MID ? ts - GF_MID : bs) : ws;
  const u64 xe = need_r ? (be - te > GF_MID ? te + GF_MID : be) : we;
  const u32 xn = (u32)(xe - xs);
  const u32 nl = (u32)(ws - xs), nr = (u32)(xe - we);  // outer halo lengths (<= XH)
  if (need_l || need_r) {
    // top bits of the outer halo: one position per thread and side
    static_assert(XH <= (u32)GF1_NT, "one outer-halo position per thread");
    const u32* const hi = reinterpret_cast<const u32*>(src) + 1;  // high words: hi[2 g]
    if (tid < nl) s_xt[0][tid] = hi[2 * (xs + tid)] >> (gsh - 32);
    if (tid < nr) s_xt[1][tid] = hi[2 * (we + tid)] >> (gsh - 32);
    __syncthreads();
  }
  // top bits of outer-window position x
  auto top = [&](u32 x) -> u32 {
    if (x < nl) return s_xt[0][x];
    const u32 i = x - nl;
    return i < wn ? (u32)(s_k[i] >> gsh) : s_xt[1][i - wn];
  };
  // Position x starts a group when it is the block's first key or its top
  // bits differ from those at x - 1; the window's first position inside a
  // block is no start (a group reaching past it counts as too large), and the
  // block's end counts as one.  One ballot per 64 positions.
  // A word inside the window without any start (a run of 64 equal top bits)
  // is noted: only then can a group's bounds lie beyond the neighbouring
  // words.  (The window's last, partial word holds position xn, whose start
  // bit is set at the block's end; otherwise a group reaching it is too large
  // either way.)
  const bool xfirst = xs == bs, xlast = xe == be;
  if (nl == 0 && nr == 0) {
    for (u32 base = 0; base < xn + 1; base += GF1_NT) {
      const u32 x = base + tid;
      bool h = false;
      if (x < xn) h = x == 0 ? xfirst : (s_k[x] >> gsh) != (s_k[x - 1] >> gsh);
      else if (x == xn) h = xlast;
      const u64 m = __ballot(h);
      if (lane == 0 && x < xn + 64) {
        s_hb[x >> 6] = m;
        if (m == 0 && x + 64 <= xn) s_empty = 1u;  // a whole word inside the window
      }
    }
  } else {
    for (u32 base = 0; base < xn + 1; base += GF1_NT) {
      const u32 x = base + tid;
      bool h = false;
      if (x < xn) h = x == 0 ? xfirst : top(x) != top(x - 1);
      else if (x == xn) h = xlast;
      const u64 m = __ballot(h);
      if (lane == 0 && x < xn + 64) {
        s_hb[x >> 6] = m;
        if (m == 0 && x + 64 <= xn) s_empty = 1u;  // a whole word inside the window
      }
    }
  }
  __syncthreads();
  // Nearest group starts per word, when some word has none: a running
  // maximum from the left and a running minimum from the right, by the
  // first wave (three words per lane).
  constexpr u32 NONE = 0xFFFFFFFFu;
  static_assert(NW <= 3 * 64, "three head-bit words per lane");
  const bool tables = s_empty != 0;
  if (tables && tid < 64) {
    u32 last[3], first[3];
    u32 run = 0;  // last start + 1 (0: none)
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      const u32 wi = tid * 3 + i;
      const u64 m = wi < NW ? s_hb[wi] : 0;
      if (m) run = wi * 64 + 64 - (u32)__clzll((long long)m);
      last[i] = run;
    }
    u32 incl = run;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
      const u32 y = __shfl_up(incl, d);
      if (tid >= (u32)d && y > incl) incl = y;
    }
    u32 prev = __shfl_up(incl, 1);
    if (tid == 0) prev = 0;
    u32 runf = NONE;  // first start
#pragma unroll
    for (int i = 2; i >= 0; --i) {
      const u32 wi = tid * 3 + i;
      const u64 m = wi < NW ? s_hb[wi] : 0;
      if (m) runf = wi * 64 + (u32)__ffsll((long long)m) - 1;
      first[i] = runf;
    }
    u32 inclf = runf;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
      const u32 y = __shfl_down(inclf, d);
      if (tid + d < 64 && y < inclf) inclf = y;
    }
    u32 nextf = __shfl_down(inclf, 1);
    if (tid == 63) nextf = NONE;
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      const u32 wi = tid * 3 + i;
      if (wi < NW) {
        const u32 l = last[i] > prev ? last[i] : prev;
        s_last[wi] = l ? l - 1 : NONE;
        s_first[wi] = first[i] < nextf ? first[i] : nextf;
      }
    }
  }
  if (tables) __syncthreads();
  // Places first (mid-size group starts gathered in LDS), then one list
  // reservation per tile, then the writes.
  bool bad = false;
  u32 place[VL];  // outer-window output position, NONE for a mid-size group's key
#pragma unroll
  for (int k = 0; k < VL; ++k) {
    place[k] = NONE;
    const u32 w = o0 + (u32)k * GF1_NT + tid;  // inner-window position
    if (w >= o1) break;
    const u32 x = w + nl;                      // outer-window position
    const u64 key = s_k[w];
    // group bounds: the last start at or before x and the first start after it
    const u32 xi = x >> 6, b = x & 63;
    const u64 upto = ((u64)2 << b) - 1;  // bits 0..b
    const u64 hb = s_hb[xi];
    const u64 mb = hb & upto, ma = hb & ~upto;
    u32 gs = NONE, ge = NONE;
    if (mb) {
      gs = xi * 64 + 63 - (u32)__clzll((long long)mb);
    } else if (xi > 0) {
      const u64 m = s_hb[xi - 1];  // not empty unless the tables were built
      gs = m ? (xi - 1) * 64 + 63 - (u32)__clzll((long long)m) : (tables ? s_last[xi - 1] : NONE);
    }
    if (ma) {
      ge = xi * 64 + (u32)__ffsll((long long)ma) - 1;
    } else if (xi + 1 < NW) {
      const u64 m = s_hb[xi + 1];
      ge = m ? (xi + 1) * 64 + (u32)__ffsll((long long)m) - 1 : (tables ? s_first[xi + 1] : NONE);
    }
    const bool whole = gs != NONE && ge != NONE && ge <= xn;
    const u32 gn = whole ? ge - gs : 0xFFFFFFFFu;
    u32 o = x;
    if (gn <= GF_HALO) {
      // inside the inner window: rank among the group by (key, position)
      u32 r = 0;
      for (u32 j = gs - nl; j < ge - nl; ++j) {
        const u64 kj = s_k[j];
        r += (kj < key || (kj == key && j < w)) ? 1u : 0u;
      }
      o = gs + r;
    } else if (gn > GF_MID && gs != x && s_k[w - 1] != key) {
      bad = true;  // a large group with different keys (w >= 1 here)
    }
    if (gn > GF_HALO && gn <= GF_MID) {
      // written by k_group_mid; listed once, by the tile holding its start
      if (x == gs) s_mid[atomicAdd(&s_nmid, 1u)] = (xs + gs) | ((u64)gn << 44);
    } else {
      place[k] = o;
    }
  }
  __syncthreads();
  const u32 nm = s_nmid;
  if (nm) {
    if (tid == 0) s_mbase = atomicAdd(&p.counters[C_NMID], nm);
    __syncthreads();
    const u32 base = s_mbase;
    for (u32 i = tid; i < nm; i += GF1_NT) {
      if ((u64)base + i < p.mid_cap) p.midlist[base + i] = s_mid[i];
      else bad = true;  // cannot happen for a list of n / (GF_HALO + 1) + 1 entries; the block is redone
    }
  }
#pragma unroll
  for (int k = 0; k < VL; ++k) {
    const u32 w = o0 + (u32)k * GF1_NT + tid;
    if (w >= o1) break;
    if (place[k] != NONE) {
      dst[xs + place[k]] = s_k[w];
      if (HASV) dstv[xs + place[k]] = v[k];
      block_sample<u64>(p, blk, bs, xs + place[k], s_k[w]);
    }
  }
  if (__ballot(bad) != 0 && lane == 0) p.gflags2[blk] = 1u;
}

template <bool HASV>
void launch_group_fix_mid(const Plan& p, const u64* src, const u32* srcv, u64* dst, u32* dstv, hipStream_t s) {
  if (p.max_tiles == 0) return;
  const int pe_ = prof_begin(s);
  hipLaunchKernelGGL(k_group_fix_mid<HASV>, dim3(p.max_tiles * (p.rtile / GF1_SPAN)), dim3(GF1_NT), 0, s, p, src, srcv, dst, dstv);
  prof_end(pe_, "group_fix_mid", s);
}
template void launch_group_fix_mid<false>(const Plan&, const u64*, const u32*, u64*, u32*, hipStream_t);
template void launch_group_fix_mid<true>(const Plan&, const u64*, const u32*, u64*, u32*, hipStream_t);

// ----------------------------------------------------------------- mid-size groups
// Groups of GF_HALO+1 .. GF_MID keys listed by k_group_fix.  Their bits from
// p.gshift up are equal, so a stable LSD sort over the digits below (five, or
// four for doubles) finishes them.
// Each wave takes whole groups (static stride over the list): the group sits
// in registers (GM_ITEMS keys per lane), every pass ranks with the wave's own
// digit counters and scatters through the wave's LDS slice.
constexpr int GM_NT = 256;
constexpr int GM_WAVES = GM_NT / 64;
constexpr int GM_ITEMS = GF_MID / 64;

// LDS accesses of one wave to its own slice, ordered across its lanes.
__device__ inline void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

template <bool HASV>
__global__ __launch_bounds__(GM_NT) void k_group_mid(Plan p, const u64* __restrict__ src,
                                                    const u32* __restrict__ srcv, u64* __restrict__ dst,
                                                    u32* __restrict__ dstv) {
  __shared__ u64 s_k[GM_WAVES][GF_MID];
  __shared__ u32 s_v[GM_WAVES][HASV ? GF_MID : 1];
  __shared__ u32 s_c[GM_WAVES][RADIX];
  __shared__ u64 s_hw[GM_WAVES][GM_ITEMS + 1];  // run-start bits of a group
  const u32 lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const u64 nmid = p.counters[C_NMID] < p.mid_cap ? p.counters[C_NMID] : p.mid_cap;
  const u32 nw = gridDim.x * GM_WAVES;
  // digits below the group shift (5, or 4 for doubles); after the pass over
  // the highest of them, runs of equal key >> rsh remain
  const u32 gd = p.gshift / RADIX_BITS, rsh = (gd - 1) * RADIX_BITS;
  u64* const sk = s_k[w];
  u32* const sv = s_v[w];
  u32* const sc = s_c[w];
  u64* const shw = s_hw[w];
  for (u64 e = blockIdx.x * GM_WAVES + w; e < nmid; e += nw) {
    const u64 ent = p.midlist[e];
    const u64 g0 = ent & ((1ull << 44) - 1);
    const u32 len = (u32)(ent >> 44) < GF_MID ? (u32)(ent >> 44) : GF_MID;
    const int nj = (int)((len + 63) / 64);
    // the group's block (for its block samples): the last block starting at
    // or before g0 (a group lies inside one non-empty block)
    u32 gblk = 0;
    u64 gbs = 0;
    if (p.bsamp) {
      gblk = find_seg(p.blk_start, p.NB, g0);
      gbs = p.blk_start[gblk];
    }
    u64 keys[GM_ITEMS];
    u32 vals[HASV ? GM_ITEMS : 1];
#pragma unroll
    for (int j = 0; j < GM_ITEMS; ++j) {
      const u32 idx = j * 64 + lane;
      keys[j] = idx < len ? src[g0 + idx] : 0;
      if (HASV) vals[j] = idx < len ? srcv[g0 + idx] : 0u;
    }
    // One stable LSD pass over digit `pass` (scatter through the wave's LDS
    // slice); left out when every key has the same digit there.
    auto radix_pass = [&](u32 pass) {
      for (u32 i = lane; i < RADIX; i += 64) sc[i] = 0;
      wave_lds_sync();
      u32 rank[GM_ITEMS], dig[GM_ITEMS];
      rank_items<u64, GM_ITEMS, u32>(keys, 0, len, pass * RADIX_BITS, sc, rank, dig, nj);
      wave_lds_sync();
      // every key has the same digit: the pass leaves the order as it is
      if (sc[__shfl(dig[0], 0)] == len) return;
      // exclusive scan of the 256 counts, four per lane
      const u32 c0 = sc[4 * lane], c1 = sc[4 * lane + 1], c2 = sc[4 * lane + 2], c3 = sc[4 * lane + 3];
      const u32 tsum = c0 + c1 + c2 + c3;
      u32 incl = tsum;
#pragma unroll
      for (int d = 1; d < 64; d <<= 1) {
        const u32 y = __shfl_up(incl, d);
        if (lane >= (u32)d) incl += y;
      }
      const u32 ex = incl - tsum;
      wave_lds_sync();
      sc[4 * lane] = ex;
      sc[4 * lane + 1] = ex + c0;
      sc[4 * lane + 2] = ex + c0 + c1;
      sc[4 * lane + 3] = ex + c0 + c1 + c2;
      wave_lds_sync();
#pragma unroll
      for (int j = 0; j < GM_ITEMS; ++j) {
        if (j >= nj) break;
        if (j * 64 + lane < len) {
          const u32 pos = sc[dig[j]] + rank[j];
          sk[pos] = keys[j];
          if (HASV) sv[pos] = vals[j];
        }
      }
      wave_lds_sync();
#pragma unroll
      for (int j = 0; j < GM_ITEMS; ++j) {
        if (j >= nj) break;
        const u32 idx = j * 64 + lane;
        if (idx < len) {
          keys[j] = sk[idx];
          if (HASV) vals[j] = sv[idx];
        }
      }
      wave_lds_sync();
    };
    // The bits from gshift up are equal in a group.  One pass over the digit
    // below them (digit 4, bits 32..39, for gshift 40) leaves runs of keys
    // with equal key >> rsh, short for keys spread over the low bits; a run
    // of at most 64 keys is finished by ranking by (key, position).  If some
    // run is longer, the passes over digits 0..gd-1 sort the group instead
    // (stable from any starting order).
    radix_pass(gd - 1);
#pragma unroll
    for (int j = 0; j < GM_ITEMS; ++j) {
      if (j >= nj) break;
      const u32 idx = j * 64 + lane;
      if (idx < len) sk[idx] = keys[j];
    }
    wave_lds_sync();
    // run starts (and the end at len), one ballot per 64 positions
#pragma unroll
    for (int j = 0; j <= GM_ITEMS; ++j) {
      if (j > nj) break;
      const u32 i = j * 64 + lane;
      const bool h = i < len ? (i == 0 || (sk[i] >> rsh) != (sk[i - 1] >> rsh)) : i == len;
      const u64 m = __ballot(h);
      if (lane == 0) shw[j] = m;
    }
    wave_lds_sync();
    u32 run[GM_ITEMS];  // run start | run end << 16
    bool longrun = false;
#pragma unroll
    for (int j = 0; j < GM_ITEMS; ++j) {
      run[j] = 0;
      if (j >= nj) break;
      const u32 i = j * 64 + lane;
      if (i < len) {
        const u64 upto = ((u64)2 << lane) - 1;  // bits 0..lane
        u64 m = shw[j] & upto;
        int wi = j;
        while (m == 0) m = shw[--wi];  // position 0 is a start
        const u32 rs = (u32)wi * 64 + 63 - (u32)__clzll((long long)m);
        m = shw[j] & ~upto;
        wi = j;
        while (m == 0) m = shw[++wi];  // position len is marked
        const u32 re = (u32)wi * 64 + (u32)__ffsll((long long)m) - 1;
        run[j] = rs | re << 16;
        longrun = longrun || re - rs > 64;
      }
    }
    if (__ballot(longrun) != 0) {
      for (u32 pass = 0; pass < gd; ++pass) radix_pass(pass);
    } else {
#pragma unroll
      for (int j = 0; j < GM_ITEMS; ++j) {
        if (j >= nj) break;
        const u32 i = j * 64 + lane;
        if (i < len) {
          const u32 rs = run[j] & 0xFFFFu, re = run[j] >> 16;
          u32 r = rs;
          for (u32 x = rs; x < re; ++x) {
            const u64 kx = sk[x];
            r += (kx < keys[j] || (kx == keys[j] && x < i)) ? 1u : 0u;
          }
          dst[g0 + r] = keys[j];
          if (HASV) dstv[g0 + r] = vals[j];
          block_sample<u64>(p, gblk, gbs, g0 + r, keys[j]);
        }
      }
      continue;
    }
#pragma unroll
    for (int j = 0; j < GM_ITEMS; ++j) {
      const u32 idx = j * 64 + lane;
      if (idx < len) {
        dst[g0 + idx] = keys[j];
        if (HASV) dstv[g0 + idx] = vals[j];
        block_sample<u64>(p, gblk, gbs, g0 + idx, keys[j]);
      }
    }
  }
}

template <bool HASV>
void launch_group_mid(const Plan& p, const u64* src, const u32* srcv, u64* dst, u32* dstv, u32 wgs, hipStream_t s) {
  if (p.max_tiles == 0 || p.mid_cap == 0) return;
  const int pe_ = prof_begin(s);
  hipLaunchKernelGGL(k_group_mid<HASV>, dim3(wgs), dim3(GM_NT), 0, s, p, src, srcv, dst, dstv);
  prof_end(pe_, "group_mid", s);
}
template void launch_group_mid<false>(const Plan&, const u64*, const u32*, u64*, u32*, u32, hipStream_t);
template void launch_group_mid<true>(const Plan&, const u64*, const u32*, u64*, u32*, u32, hipStream_t);

// ----------------------------------------------------------------- small blocks
// A block of at most one tile is sorted entirely in LDS: all digit passes,
// no look-back, one read and one write of global memory.
template <typename K, bool HASV>
__global__ __launch_bounds__(SORT_NT) void k_small_sort(Plan p, const K* __restrict__ src,
                                                        const u32* __restrict__ srcv, K* __restrict__ dst,
                                                        u32* __restrict__ dstv) {
  constexpr int NWV = SORT_NT / 64, WI = 64 * SORT_ITEMS;
  constexpr int D = KeyT<K>::BITS / RADIX_BITS;
  __shared__ u32 s_wc[NWV][RADIX];
  __shared__ u32 s_lstart[RADIX];
  __shared__ u64 s_scan[NWV];
  __shared__ K s_keys[SMALL_TILE];
  __shared__ u32 s_vals[HASV ? SMALL_TILE : 1];
  const u32 tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  if (blockIdx.x >= p.counters[C_NSMALL]) return;
  const u32 blk = p.small_list[blockIdx.x];
  const u64 bstart = p.blk_start[blk];
  const u32 n = (u32)(p.blk_start[blk + 1] - bstart);
  const u32 wbase = w * WI;
  K keys[SORT_ITEMS];
  u32 vals[HASV ? SORT_ITEMS : 1];
  if (!HASV || srcv != nullptr) {
#pragma unroll
    for (int j = 0; j < SORT_ITEMS; ++j) {
      const u32 idx = wbase + j * 64 + lane;
      keys[j] = idx < n ? src[bstart + idx] : (K)0;
      if (HASV) vals[j] = idx < n ? srcv[bstart + idx] : 0u;
    }
  } else {
    // no value array: the values are the keys' input positions inside their instance
    const u64 vgen = bstart - p.seg[blk / p.P];
#pragma unroll
    for (int j = 0; j < SORT_ITEMS; ++j) {
      const u32 idx = wbase + j * 64 + lane;
      keys[j] = idx < n ? src[bstart + idx] : (K)0;
      if (HASV) vals[j] = (u32)(vgen + idx);
    }
  }
  if ((p.kx_top | p.kx_fm) != 0) {
#pragma unroll
    for (int j = 0; j < SORT_ITEMS; ++j) keys[j] = key_in<K>(keys[j], p.kx_top, p.kx_fm);
  }
  for (int pass = 0; pass < D; ++pass) {
    const u32 shift = pass * RADIX_BITS;
    for (int i = tid; i < NWV * RADIX; i += SORT_NT) (&s_wc[0][0])[i] = 0;
    __syncthreads();
    u32 rank[SORT_ITEMS], dig[SORT_ITEMS];
    rank_items<K, SORT_ITEMS, u32>(keys, wbase, n, shift, s_wc[w], rank, dig);
    __syncthreads();
    u32 tot = 0;
#pragma unroll
    for (int v = 0; v < NWV; ++v) {
      const u32 c = s_wc[v][tid];
      s_wc[v][tid] = tot;
      tot += c;
    }
    u64 ttot;
    s_lstart[tid] = (u32)block_exclusive_scan<SORT_NT>(tot, s_scan, ttot);
    __syncthreads();
#pragma unroll
    for (int j = 0; j < SORT_ITEMS; ++j) {
      if (wbase + j * 64 + lane < n) {
        const u32 pos = s_lstart[dig[j]] + s_wc[w][dig[j]] + rank[j];
        s_keys[pos] = keys[j];
        if (HASV) s_vals[pos] = vals[j];
      }
    }
    __syncthreads();
    if (pass + 1 < D) {
#pragma unroll
      for (int j = 0; j < SORT_ITEMS; ++j) {
        const u32 idx = wbase + j * 64 + lane;
        keys[j] = idx < n ? s_keys[idx] : (K)0;
        if (HASV) vals[j] = idx < n ? s_vals[idx] : 0u;
      }
      __syncthreads();
    }
  }
  for (u32 i = tid; i < n; i += SORT_NT) {
    dst[bstart + i] = s_keys[i];
    if (HASV) dstv[bstart + i] = s_vals[i];
    block_sample<K>(p, blk, bstart, bstart + i, s_keys[i]);
  }
}

// ----------------------------------------------------------------- launchers
void launch_plan(const Plan& p, hipStream_t s) {
  { const int pe_ = prof_begin(s); hipLaunchKernelGGL(k_plan, dim3(1), dim3(1024), 0, s, p); prof_end(pe_, p.only ? "plan_fallback" : "plan", s); }
  if (p.max_tiles) {
    const int pe_ = prof_begin(s);
    hipLaunchKernelGGL(k_tile_desc, dim3((p.max_tiles + 255) / 256), dim3(256), 0, s, p);
    prof_end(pe_, p.only ? "tile_desc_fallback" : "tile_desc", s);
  }
}

void launch_fill_set(const FillSet& f, hipStream_t s) {
  u64 most = 0;
  for (int r = 0; r < f.count; ++r) most = f.n[r] > most ? f.n[r] : most;
  if (most == 0) return;
  u64 blocks = (most + 255) / 256;
  if (blocks > 8192) blocks = 8192;
  { const int pe_ = prof_begin(s); hipLaunchKernelGGL(k_fill_set, dim3((u32)blocks), dim3(256), 0, s, f); prof_end(pe_, "fill", s); }
}

template <typename K>
void launch_hist(const Plan& p, const K* src, hipStream_t s, u32 dlo) {
  if (p.max_tiles == 0) return;
  // tiles per workgroup: up to HIST_TILES, but at least a few workgroups per compute unit
  u32 tpw = p.max_tiles / p.persist_wgs;
  tpw = tpw < 1 ? 1 : (tpw > HIST_TILES ? HIST_TILES : tpw);
  { const int pe_ = prof_begin(s); if (sizeof(K) == 8 && dlo == 5)
      hipLaunchKernelGGL((k_hist<K, 5>), dim3((p.max_tiles + tpw - 1) / tpw), dim3(SORT_NT), 0, s, p, src, tpw);
    else if (sizeof(K) == 8 && dlo == 4)
      hipLaunchKernelGGL((k_hist<K, 4>), dim3((p.max_tiles + tpw - 1) / tpw), dim3(SORT_NT), 0, s, p, src, tpw);
    else
      hipLaunchKernelGGL((k_hist<K, 0>), dim3((p.max_tiles + tpw - 1) / tpw), dim3(SORT_NT), 0, s, p, src, tpw); prof_end(pe_, p.only ? "hist_fallback" : "hist", s); }
  const u32 waves = p.NB * p.D;
  { const int pe_ = prof_begin(s); hipLaunchKernelGGL(k_scan_hist, dim3((waves + 3) / 4), dim3(256), 0, s, p); prof_end(pe_, p.only ? "scan_hist_fallback" : "scan_hist", s); }
}

template <typename K, bool HASV>
void launch_presorted(const Plan& p, const K* src, const u32* srcv, K* dst, u32* dstv, hipStream_t s) {
  if (p.max_tiles == 0) return;
  const int pe_ = prof_begin(s);
  hipLaunchKernelGGL((k_presorted<K, HASV>), dim3((p.max_tiles + PRESORTED_TPW - 1) / PRESORTED_TPW), dim3(256), 0, s, p,
                     src, srcv, dst, dstv);
  prof_end(pe_, "presorted", s);
}

template <typename K, bool HASV>
void launch_small_sort(const Plan& p, const K* src, const u32* srcv, K* dst, u32* dstv, hipStream_t s) {
  { const int pe_ = prof_begin(s); hipLaunchKernelGGL((k_small_sort<K, HASV>), dim3(p.NB), dim3(SORT_NT), 0, s, p, src, srcv, dst, dstv); prof_end(pe_, "small_sort", s); }
}

template <typename K, bool HASV>
void launch_onesweep(const Plan& p, const K* src, const u32* srcv, K* dst, u32* dstv, u32 pass, hipStream_t s) {
  if (p.max_tiles == 0) return;
  // Persistent grid: tiles of 4096 keys take 512-thread workgroups with 8
  // keys per thread, tiles of 8192 keys 512-thread workgroups with 16 keys
  // per thread (two workgroups per compute unit: at most 80 KB of LDS each),
  // except 64-bit keys with values, whose tiles of 8192 take one 1024-thread
  // workgroup per compute unit with 8 keys and 8 values per thread (measured
  // faster than loading the values in a second phase), and tiles of 16384
  // 32-bit keys take one 1024-thread workgroup with 16 keys per thread; a
  // multiple of the queue count.
  constexpr bool WIDE_PAIRS = sizeof(K) == 8 && HASV;
  const u32 NT = p.rtile == RTILE_HUGE || (WIDE_PAIRS && p.rtile == RTILE_LARGE) ? 1024 : 512;
  u32 grid = p.persist_wgs * 256 / NT;
  grid = grid < p.max_tiles ? grid : p.max_tiles;
  grid = (grid + p.nq - 1) / p.nq * p.nq;
  const int pe_ = prof_begin(s);
  if constexpr (sizeof(K) == 4) {
    if (p.rtile == RTILE_HUGE) {
      if (p.only)
        hipLaunchKernelGGL((k_onesweep<K, HASV, 1024, 16, 1, true>), dim3(grid), dim3(NT), 0, s, p, src, srcv, dst, dstv,
                           pass);
      else
        hipLaunchKernelGGL((k_onesweep<K, HASV, 1024, 16, 1, false>), dim3(grid), dim3(NT), 0, s, p, src, srcv, dst,
                           dstv, pass);
      prof_end(pe_, p.only ? "onesweep_fallback" : "onesweep", s);
      return;
    }
  }
  if (p.rtile == RTILE_SMALL) {
    if (p.only)
      hipLaunchKernelGGL((k_onesweep<K, HASV, RTILE_SMALL / 8, 8, 2, true>), dim3(grid), dim3(NT), 0, s, p, src, srcv,
                         dst, dstv, pass);
    else
      hipLaunchKernelGGL((k_onesweep<K, HASV, RTILE_SMALL / 8, 8, 2, false>), dim3(grid), dim3(NT), 0, s, p, src, srcv,
                         dst, dstv, pass);
  } else if constexpr (WIDE_PAIRS) {
    if (p.only)
      hipLaunchKernelGGL((k_onesweep<K, HASV, RTILE_LARGE / 8, 8, 1, true>), dim3(grid), dim3(NT), 0, s, p, src, srcv,
                         dst, dstv, pass);
    else
      hipLaunchKernelGGL((k_onesweep<K, HASV, RTILE_LARGE / 8, 8, 1, false>), dim3(grid), dim3(NT), 0, s, p, src, srcv,
                         dst, dstv, pass);
  } else {
    if (p.only)
      hipLaunchKernelGGL((k_onesweep<K, HASV, RTILE_LARGE / 16, 16, 4, true>), dim3(grid), dim3(NT), 0, s, p, src, srcv,
                         dst, dstv, pass);
    else
      hipLaunchKernelGGL((k_onesweep<K, HASV, RTILE_LARGE / 16, 16, 4, false>), dim3(grid), dim3(NT), 0, s, p, src, srcv,
                         dst, dstv, pass);
  }
  prof_end(pe_, p.only ? "onesweep_fallback" : "onesweep", s);
}

#define LBS_INST(K)                                                                                     \
  template void launch_hist<K>(const Plan&, const K*, hipStream_t, u32);                                   \
  template void launch_presorted<K, false>(const Plan&, const K*, const u32*, K*, u32*, hipStream_t);  \
  template void launch_presorted<K, true>(const Plan&, const K*, const u32*, K*, u32*, hipStream_t);   \
  template void launch_small_sort<K, false>(const Plan&, const K*, const u32*, K*, u32*, hipStream_t); \
  template void launch_small_sort<K, true>(const Plan&, const K*, const u32*, K*, u32*, hipStream_t);  \
  template void launch_onesweep<K, false>(const Plan&, const K*, const u32*, K*, u32*, u32, hipStream_t); \
  template void launch_onesweep<K, true>(const Plan&, const K*, const u32*, K*, u32*, u32, hipStream_t);
LBS_INST(u32)
LBS_INST(u64)
#undef LBS_INST

}  // namespace lbs
