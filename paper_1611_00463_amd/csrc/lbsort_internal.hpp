// Internal definitions shared by the kernels and the engine of lbsort.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

namespace lbs {

typedef uint32_t u32;
typedef uint64_t u64;

// Radix sort geometry (step 1): 8-bit digits.  Blocks of at most SMALL_TILE
// keys are sorted whole in LDS (SORT_NT threads x SORT_ITEMS keys); larger
// blocks are cut into radix tiles of Plan::rtile keys, RTILE_SMALL,
// RTILE_LARGE or (32-bit keys) RTILE_HUGE (a call's choice, the same for all
// its passes).
constexpr int RADIX_BITS = 8;
constexpr int RADIX = 1 << RADIX_BITS;
constexpr int SORT_NT = 256;
constexpr int SORT_ITEMS = 16;
constexpr int SMALL_TILE = SORT_NT * SORT_ITEMS;  // 4096 keys
constexpr u32 RTILE_SMALL = 4096;
constexpr u32 RTILE_LARGE = 8192;
constexpr u32 RTILE_HUGE = 16384;  // 32-bit keys only (the staged tile fills most of the LDS)
constexpr int WAVE = 64;
// Group fix-up of the 64-bit local sort: groups of at most GF_HALO keys are
// ranked in place; in the blocks that have larger groups of different keys,
// groups of up to GF_MID keys are listed (at most n / (GF_HALO + 1) of them)
// and sorted by a second kernel.
constexpr u32 GF_HALO = 64;
constexpr u32 GF_MID = 512;

// Look-back status word: [63:56] epoch (pass + 1), [55:54] flag, [53:0] count.
constexpr u64 ST_AGG = 1, ST_INC = 2;
constexpr u64 ST_VALMASK = (1ull << 54) - 1;
__host__ __device__ inline u64 st_pack(u32 epoch, u64 flag, u64 v) {
  return ((u64)epoch << 56) | (flag << 54) | (v & ST_VALMASK);
}

// Slots of the small counter array at the head of the workspace.
constexpr int NQ = 8;  // radix tile queues, one per XCD of the MI355X
enum Counter : int {
  C_ERR = 0,        // device error bits (sticky until lbsort_check)
  C_NSMALL = 1,     // number of blocks sorted whole in LDS
  C_NLARGE = 2,     // blocks larger than one tile
  C_NMID = 3,       // groups listed for the mid-size group sort
  C_ANYFLAG = 4,    // some block was flagged by the group fix-up
  C_RUN_TOP = 5,    // bit j: digit j takes two or more values in some large block (top-digit passes)
  C_RUN_REDO = 6,   // the same over the blocks of the fallback plan
  C_QPARAM = 8,     // C_QPARAM + 4x + {0: blocks, 1: rmin, 2: first status slot, 3: tiles} of queue x
  C_TICKET = 64,    // C_TICKET + NQ * pass + x: next ticket of queue x in radix pass `pass`
  C_COUNT = 128
};
enum DevErr : u32 {
  E_SPIN = 1u,         // a decoupled look-back wait gave up
  E_SEG = 2u,          // malformed segment table
  E_SELECT = 4u,       // merge-path selection did not converge
  E_RANGE = 8u         // an instance or block too large for 32-bit counters
};

// One radix tile of a queue, resolved once per call (the mapping from a
// queue's tickets to blocks and tiles is the same in every digit pass).
struct TileDesc {
  u64 bstart;  // first key of the tile's block
  u64 tbase;   // first key of the tile
  u32 blk;     // block index
  u32 lt;      // tile index inside the block
  u32 jx;      // block index inside the queue
  u32 tile_n;  // keys in the tile
  u32 tail;    // ticket of the block's tile u >= rmin is tail + u (mod 2^32)
  u32 pad;
};

// Everything a kernel needs to know about one call, passed by value.
struct Plan {
  u32 B, P, NB;          // instances, processors, blocks = B * P
  u32 s;                 // samples per block (before capping by block size)
  u32 D;                 // radix passes = key bits / 8
  u32 inv;               // investigator mode
  u32 F, L, TM;          // merge fan-in, merge levels, merge tile
  u32 max_tiles;         // radix tiles, worst case
  u32 rtile;             // keys per radix tile: RTILE_SMALL, RTILE_LARGE or RTILE_HUGE
  u32 nq;                // radix tile queues (NQ, or 1)
  u32 persist_wgs;       // workgroups of the persistent radix pass
  u64 total_n;
  const u64* seg;        // [B+1]
  u64* blk_start;        // [NB+1]
  u32* tstart;           // [NB+1] radix tile prefix (blocks larger than one tile)
  u32* small_list;       // [NB]
  u32* large_list;       // [NB] blocks larger than one tile, in block order
  u32* rem_prefix;       // [NB+1] over large blocks: prefix of (tiles - C_RMIN)
  TileDesc* tdesc;       // [max_tiles] by status slot (queue base + ticket)
  const u32* only;       // [NB] or null: plan only the large blocks with only[b] != 0
  const u32* skip;       // [NB] or null: leave out the large blocks with skip[b] != 0
  u32* presorted;        // [NB] or null: bit 0 = the block is non-decreasing, bit 1 =
                         // non-increasing (set to 3 before k_hist, which clears bits)
  u32 epoch_base;        // added to the look-back epochs of the radix passes
  u32* gflags;           // [NB] blocks the group fix-up could not finish
  u32* gflags2;          // [NB] blocks the mid-size group fix-up could not finish either
  u64* midlist;          // [mid_cap] groups of 65..GF_MID keys: start | length << 44
  u64 mid_cap;           // entries of midlist (0: no list)
  u32* counters;         // [C_COUNT]
  u32* hist;             // [NB][D][256]
  u64* status;           // [max_tiles][256]
  u64* samp_start;       // [NB+1]
  void* samples;         // [<= NB*s] keys
  void* pool;            // [<= NB*s] keys, sample pool sorted per instance
  u64* lo;               // [B][P][P-1]
  u64* hi;               // [B][P][P-1]
  u64* cuts;             // [B][P][P+1]
  u64* Dm;               // [B][P+1][P] receive offsets, row P = G_{k+1}
  u64* G;                // [B][P+1]
  void* splitters;       // [B][P-1]
  u32* mtile;            // [NGmax+1] merge tile prefix of the current level
  u64* rec_start;        // [mtiles][F] per merge tile: first source element of each run
  u64* rec_end;          // [mtiles][F] per merge tile: one past the last
  u64* rec_out;          // [mtiles]    per merge tile: first output position
  u32* rec_n;            // [mtiles]    per merge tile: element count
  u32* slot_grp;         // [mtiles+NGmax] merge boundary slot -> group
  u64* grp_run;          // [NGmax][F][2] per group and input run: source offset, length
  u64* grp_out;          // [NGmax][2]    per group: output offset, length
  u32 ng_max;            // merge groups, worst case over levels
  u32 mtiles_max;        // merge tiles, worst case over levels
  // Keys of signed and floating-point types are sorted as unsigned integers
  // through an order-preserving map (key_in), undone where keys leave the
  // library (key_out).  Both are zero (the identity) except in the plan
  // copies of the launches that read the caller's keys or write them back.
  u64 kx_top, kx_fm;     // map applied to keys read from keys_in
  u64 ky_top, ky_fm;     // inverse applied to keys written to keys_out / splitters
  u32 vidx;              // values are generated: input position inside the instance
  // Digit passes that may be left out (run_slot != 0): k_scan_hist sets bit j
  // of counters[run_slot] when digit j takes two or more values in some
  // block; a pass of run_mask whose bit is clear leaves every block as it is
  // and does not run (the highest pass of run_mask runs when no bit is set).
  // The passes that run read the input first and then alternate between
  // pass_out and pass_tmp so that the last one writes pass_out.
  u32 run_slot, run_mask;
  void* pass_out;
  u32* pass_outv;
  void* pass_tmp;
  u32* pass_tmpv;
  // Block samples for the one-pass handler (null otherwise): every kernel
  // that writes the local sort's final output also writes the key at each
  // block position x = 0, m, 2m, ... to bsamp[floor(bstart / m) + block +
  // x / m] (block_sample), so that the handler's samples need no strided
  // read of the sorted blocks.
  void* bsamp;
  // The 64-bit fix-up path's group shift: the top-digit passes sort the
  // blocks by key >> gshift (40: the three top digits; 32 for doubles, whose
  // sign and exponent leave few distinct values in the top 24 bits: four),
  // and the group fix-ups finish the groups of equal key >> gshift.
  u32 gshift;
};

// The one-pass handler's sample problem (kernels_sampled.hip): the samples of
// every run, laid out like the main problem's blocks, cut matrix and range
// table, plus per partition (group g = instance * P + k) the start of its
// sorted samples and its number of merge tiles.
struct SampPlan {
  u64* sseg;      // [B+1]  sample instance starts
  u64* sbs;       // [NB+1] sample block starts
  u64* scuts;     // [B][P][P+1] sample cuts per block
  u64* sDm;       // [B][P+1][P] sample receive offsets (row P: partition ends)
  u64* gsbase;    // [NB] first sorted sample of each partition
  u32* ntile;     // [NB] merge tiles of each partition
  void* skeys[2]; // sample keys, gathered (0) and merged (ping-pong)
  u32* svals[2];  // their positions in the sorted blocks
  u32 m;          // sample stride inside a run
  u32 q;          // sorted samples per merge tile
};
constexpr u32 SAMP_STRIDE = 16;

// ----------------------------------------------------------------- helpers
template <typename K>
struct KeyT;
template <>
struct KeyT<u32> {
  static constexpr int BITS = 32;
  static constexpr u32 MAXV = 0xFFFFFFFFu;
};
template <>
struct KeyT<u64> {
  static constexpr int BITS = 64;
  static constexpr u64 MAXV = ~0ull;
};

// The order-preserving map of a key type onto unsigned integers of the same
// width: x ^ (top | (sign mask of x & fm)).  Unsigned: top = fm = 0.  Two's
// complement: top = sign bit, fm = 0 (the sign bit flipped).  IEEE binary
// floats: top = sign bit, fm = all other bits, so non-negative numbers get
// their sign bit set and negative ones are complemented; unsigned order of the
// images is then IEEE 754 totalOrder.  key_out inverts it: the sign of the
// image decides which of the two cases the key came from.
template <typename K>
__device__ inline K sign_mask(K x) {
  if constexpr (sizeof(K) == 8) return (K)((int64_t)x >> 63);
  else return (K)((int32_t)x >> 31);
}
template <typename K>
__device__ inline K key_in(K x, u64 top, u64 fm) {
  return x ^ ((K)top | (sign_mask<K>(x) & (K)fm));
}
template <typename K>
__device__ inline K key_out(K y, u64 top, u64 fm) {
  return y ^ ((K)top | (sign_mask<K>((K)~y) & (K)fm));
}

__device__ inline u32 lane_id() { return __builtin_amdgcn_mbcnt_hi(~0u, __builtin_amdgcn_mbcnt_lo(~0u, 0)); }

// Number of set bits of `mask` in lanes below the calling lane.
__device__ inline u32 count_below(u64 mask) {
  return __builtin_amdgcn_mbcnt_hi((u32)(mask >> 32), __builtin_amdgcn_mbcnt_lo((u32)mask, 0));
}

// A value every lane of the wave holds, moved to scalar registers.
__device__ inline u64 uniform_u64(u64 v) {
  return ((u64)__builtin_amdgcn_readfirstlane((u32)(v >> 32)) << 32) | __builtin_amdgcn_readfirstlane((u32)v);
}

__device__ inline void set_error(u32* counters, u32 bits) { atomicOr(&counters[C_ERR], bits); }

__device__ inline u64 ld_acquire_agent(const u64* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ inline void st_release_agent(u64* p, u64 v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Largest b in [0, n) with prefix[b] <= t (prefix non-decreasing, prefix[0] = 0).
template <typename T>
__device__ inline u32 find_seg(const T* prefix, u32 n, u64 t) {
  u32 lo = 0, hi = n;  // answer in [lo, hi)
  while (hi - lo > 1) {
    u32 mid = (lo + hi) >> 1;
    if ((u64)prefix[mid] <= t) lo = mid; else hi = mid;
  }
  return lo;
}

// find_seg by a whole wave (all 64 lanes active, the same t in each): every
// round the lanes probe 64 evenly spaced starts of the range [lo, hi) and one
// ballot of the non-decreasing test narrows it to one step, so 32768
// segments take 3 dependent loads instead of 15.
template <typename T>
__device__ inline u32 wave_find_seg(const T* prefix, u32 n, u64 t) {
  const u32 lane = threadIdx.x & 63;
  u32 lo = 0, hi = n;  // answer in [lo, hi)
  while (hi - lo > 1) {
    const u32 step = (hi - lo + 63) / 64;
    const u32 pos = lo + (lane + 1) * step;  // < hi + 64 <= n + 64
    const bool le = pos < hi && (u64)prefix[pos] <= t;
    const u32 c = (u32)__popcll(__ballot(le));  // the probes at or before the answer
    const u32 nhi = lo + (c + 1) * step;
    lo += c * step;
    hi = nhi < hi ? nhi : hi;
  }
  return lo;
}

// x of lane `l` (the same l in every lane), read without LDS.
__device__ inline u32 lane_value(u32 x, int l) { return (u32)__builtin_amdgcn_readlane((int)x, l); }
__device__ inline u64 lane_value(u64 x, int l) {
  return ((u64)lane_value((u32)(x >> 32), l) << 32) | lane_value((u32)x, l);
}

// find_seg for every thread of a workgroup whose thread i asks for x0 + i
// (x <= xlast for the threads that ask at all): two threads search for x0 and
// xlast over all n segments, every thread then only between those two (a few
// steps in place of log2 n dependent loads per thread).  s_rng: two words of
// LDS.  Called by every thread of the workgroup (it has a barrier).
template <typename T>
__device__ inline u32 wg_find_seg(const T* prefix, u32 n, u64 x, u64 x0, u64 xlast, u32* s_rng) {
  if (threadIdx.x == 0) s_rng[0] = find_seg(prefix, n, x0);
  if (threadIdx.x == 1) s_rng[1] = find_seg(prefix, n, xlast);
  __syncthreads();
  u32 lo = s_rng[0], hi = s_rng[1] + 1;  // answer in [lo, hi)
  while (hi - lo > 1) {
    const u32 mid = (lo + hi) >> 1;
    if ((u64)prefix[mid] <= x) lo = mid; else hi = mid;
  }
  return lo;
}

// Number of elements of sorted a[0, n) that are < x (lower) or <= x (upper).
template <typename K, bool UPPER>
__device__ inline u64 bsearch_count(const K* a, u64 lo, u64 hi, K x) {
  while (lo < hi) {
    u64 mid = lo + ((hi - lo) >> 1);
    K v = a[mid];
    bool go_right = UPPER ? (v <= x) : (v < x);
    if (go_right) lo = mid + 1; else hi = mid;
  }
  return lo;
}

// Block of instance b, processor i: start = seg[b] + floor(i * n_b / P).
__device__ inline u64 block_begin(const u64* seg, u32 b, u32 i, u32 P) {
  const u64 a = seg[b], n = seg[b + 1] - seg[b];
  // i <= P <= 1024: below 2^53 keys the product fits 64 bits (a 128-bit
  // division is a long software loop)
  if (n < (1ull << 53)) return a + (u64)i * n / P;
  return a + (u64)(((unsigned __int128)i * n) / P);
}

// Order of the radix tiles.  Large block j (in block order) belongs to queue
// j % nq at index jx = j / nq; each queue has its own ticket counter and is
// meant to be served by the workgroups of one XCD, so that a block's tiles,
// its look-back chain and the partial cache lines of its scattered writes
// stay in one L2.  Inside a queue, the first rmin tiles of its blocks are
// interleaved (id = lt * nblocks + jx) so that the tiles in flight belong to
// many blocks and every look-back chain stays short; the remaining tiles
// follow block by block.
struct TileQueue {
  u32 x, nq, nb, rmin;       // queue, queue count, blocks in queue, min tiles
  const u32* rem_prefix;     // indexed by global large index x + nq * jx
  __device__ inline u32 rem(u32 jx) const { return rem_prefix[x + nq * jx]; }
  __device__ inline void locate(u32 id, u32& jx, u32& lt) const {
    const u32 head = nb * rmin;
    if (id < head) {
      jx = id % nb;
      lt = id / nb;
    } else {
      const u32 y = id - head;
      u32 lo = 0, hi = nb;
      while (hi - lo > 1) {
        const u32 mid = (lo + hi) >> 1;
        if (rem(mid) <= y) lo = mid; else hi = mid;
      }
      jx = lo;
      lt = rmin + (y - rem(jx));
    }
  }
  __device__ inline u32 id_of(u32 jx, u32 lt) const {
    return lt < rmin ? lt * nb + jx : nb * rmin + rem(jx) + (lt - rmin);
  }
};

// Ranges of 32-bit words to set in one launch.
// The block sample of a key written to global position g of block blk
// (starting at bs): kept when g - bs is a multiple of SAMP_STRIDE.
template <typename K>
__device__ inline void block_sample(const Plan& p, u32 blk, u64 bs, u64 g, K key) {
  const u64 x = g - bs;
  if (p.bsamp && (x % SAMP_STRIDE) == 0) ((K*)p.bsamp)[bs / SAMP_STRIDE + blk + x / SAMP_STRIDE] = key;
}

constexpr int FILL_MAX = 6;
struct FillSet {
  u32* a[FILL_MAX];
  u64 n[FILL_MAX];
  u32 v[FILL_MAX];
  int count = 0;
  void add(u32* p, u64 words, u32 value) {
    if (words == 0) return;
    a[count] = p;
    n[count] = words;
    v[count] = value;
    ++count;
  }
};

// Search index over n sorted keys: level l >= 1 holds the keys at positions
// i * 16^l (the first key of every group of 16^l), n_l = ceil(n_{l-1} / 16)
// of them, up to the first level of at most 16 keys; level 0 is the sorted
// array itself.  Levels 1.. are stored one after another, each starting on a
// 128-byte boundary.  Laid out on the host and passed to the kernels by
// value (a level number is the same in every lane, so its fields are read
// with scalar loads).
constexpr u32 SI_FAN = 16;
constexpr int SI_MAX_LEVELS = 16;  // 16^16 = 2^64
struct SearchIndexLayout {
  int top = 0;                   // the top level (0 when n <= 16: no index)
  u64 n[SI_MAX_LEVELS + 1];      // keys per level (n[0] = n)
  u64 off[SI_MAX_LEVELS + 1];    // byte offset of level l >= 1 in the index
  u64 bytes = 0;
  SearchIndexLayout(u64 keys, u32 key_bytes) {
    n[0] = keys;
    off[0] = 0;
    u64 at = 0;
    while (n[top] > SI_FAN) {
      ++top;
      n[top] = (n[top - 1] + SI_FAN - 1) / SI_FAN;
      off[top] = at;
      at += (n[top] * key_bytes + 127) / 128 * 128;
    }
    bytes = at;
  }
};

// Optional per-launch event timing (lbsort_profile_enable).
int prof_begin(hipStream_t s);
void prof_end(int id, const char* name, hipStream_t s);

}  // namespace lbs
