// Steps 5 and 6 of Section IV on the GPU: the exchange and the handler merge.
//
// Partition k receives one sorted run from every block (block i's cut slice
// [c[i][k], c[i][k+1]) of its sorted data).  The handler of Fig. 2 merges runs
// pairwise in rounds (1->0, 3->2, ...; then 2->0, 6->4; ...), ties going to the
// lower run, which keeps the sort stable.  Here one pass over the data merges
// F runs at once (F = 2 is the paper's tree level by level; F = 4, 8, 16 do
// log2(F) of its rounds per pass inside LDS), so P runs take ceil(log_F P)
// passes.  The exchange is not a separate copy: the first merge pass reads
// the cut slices straight from the sorted blocks, and every pass writes to the
// receive offsets of the range table (D[i][k] = G_k + sum_{i'<i} C[i'][k]).
//
// Each pass cuts its output into tiles of TM elements.  The split of a tile
// boundary among the F runs is found by a wave-wide multi-pivot selection
// (k_partition); a workgroup then loads the tile's F slices into LDS and runs
// the pairwise merge tree there (k_merge).
#include "lbsort_internal.hpp"
#include "select.hpp"

namespace lbs {

struct Level {
  u32 level;  // 0-based pass
  u32 RS;     // blocks per input run  = F^level
  u32 GS;     // blocks per output run = F^(level+1)
  u32 Q;      // groups (output runs) per partition = ceil(P / GS)
  u32 NG;     // groups in all = B * P * Q
};

__device__ inline void group_info(const Plan& p, const Level& L, u32 gidx, u64& out_off, u64& out_len) {
  const u32 g = gidx % L.Q, bk = gidx / L.Q, k = bk % p.P, b = bk / p.P;
  const u32 i0 = g * L.GS, i1 = min(i0 + L.GS, p.P);
  const u64* Db = p.Dm + (u64)b * (p.P + 1) * p.P;
  out_off = p.seg[b] + Db[(u64)i0 * p.P + k];
  out_len = Db[(u64)i1 * p.P + k] - Db[(u64)i0 * p.P + k];
}

// Input run r of group gidx: element offset in the pass's source buffer and length.
__device__ inline void run_info(const Plan& p, const Level& L, u32 gidx, u32 r, u64& off, u64& len) {
  const u32 g = gidx % L.Q, bk = gidx / L.Q, k = bk % p.P, b = bk / p.P;
  const u32 i0 = g * L.GS + r * L.RS;
  if (i0 >= p.P) {
    off = 0;
    len = 0;
    return;
  }
  if (L.level == 0) {
    const u64* c = p.cuts + ((u64)b * p.P + i0) * (p.P + 1);
    off = p.blk_start[b * p.P + i0] + c[k];
    len = c[k + 1] - c[k];
  } else {
    const u32 i1 = min(i0 + L.RS, p.P);
    const u64* Db = p.Dm + (u64)b * (p.P + 1) * p.P;
    off = p.seg[b] + Db[(u64)i0 * p.P + k];
    len = Db[(u64)i1 * p.P + k] - Db[(u64)i0 * p.P + k];
  }
  // keep the run inside its instance whatever the metadata says
  const u64 lim = p.seg[b + 1];
  if (off > lim) off = lim;
  if (len > lim - off) len = lim - off;
}

// Tile counts of every group of this pass, prefix-summed (single workgroup;
// each thread takes GPT consecutive groups per round, their loads issued
// together).
__global__ __launch_bounds__(1024) void k_merge_plan(Plan p, Level L) {
  constexpr u32 GPT = 8;
  __shared__ u64 s_w[16];
  const u32 tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  u64 carry = 0;
  for (u32 base = 0; base < L.NG; base += 1024 * GPT) {
    const u32 g0 = base + tid * GPT;
    u64 nt[GPT];
#pragma unroll
    for (u32 i = 0; i < GPT; ++i) {
      nt[i] = 0;
      if (g0 + i < L.NG) {
        u64 off, len;
        group_info(p, L, g0 + i, off, len);
        nt[i] = (len + p.TM - 1) / p.TM;
      }
    }
    u64 mine = 0;
#pragma unroll
    for (u32 i = 0; i < GPT; ++i) mine += nt[i];
    u64 x = mine;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
      u64 y = __shfl_up(x, o);
      if (lane >= (u32)o) x += y;
    }
    if (lane == 63) s_w[w] = x;
    __syncthreads();
    if (w == 0) {
      u64 t = lane < 16 ? s_w[lane] : 0;
#pragma unroll
      for (int o = 1; o < 16; o <<= 1) {
        u64 y = __shfl_up(t, o);
        if (lane >= (u32)o) t += y;
      }
      if (lane < 16) s_w[lane] = t;
    }
    __syncthreads();
    u64 ex = carry + (w ? s_w[w - 1] : 0) + x - mine;
#pragma unroll
    for (u32 i = 0; i < GPT; ++i) {
      if (g0 + i < L.NG) p.mtile[g0 + i] = (u32)ex;
      ex += nt[i];
    }
    carry += s_w[15];
    __syncthreads();
  }
  if (tid == 0) p.mtile[L.NG] = (u32)carry;
}

// The owner group of every boundary slot (group g owns slots [mtile[g] + g,
// mtile[g+1] + g + 1)): one thread per slot, a binary search over the groups.
// Also the group descriptors, one thread per (group, run), so that a
// boundary's wave starts with independent loads only.
__global__ __launch_bounds__(256) void k_slot_grp(Plan p, Level L, u32 slots) {
  const u32 q = blockIdx.x * 256 + threadIdx.x;
  for (u64 x = q; x < (u64)L.NG * p.F; x += (u64)gridDim.x * 256) {
    const u32 g = (u32)(x / p.F), r = (u32)(x % p.F);
    u64 ro, rl;
    run_info(p, L, g, r, ro, rl);
    p.grp_run[2 * x] = ro;
    p.grp_run[2 * x + 1] = rl;
    if (r == 0) {
      u64 off, len;
      group_info(p, L, g, off, len);
      p.grp_out[2 * (u64)g] = off;
      p.grp_out[2 * (u64)g + 1] = len;
    }
  }
  if (q >= slots || q >= p.mtile[L.NG] + L.NG) return;
  u32 lo = 0, hi = L.NG;  // the last g with mtile[g] + g <= q
  while (hi - lo > 1) {
    const u32 mid = (lo + hi) >> 1;
    if (p.mtile[mid] + mid <= q) lo = mid; else hi = mid;
  }
  p.slot_grp[q] = lo;
}

// One wave per tile boundary.  Group g owns boundary slots
// [mtile[g] + g, mtile[g+1] + g + 1): boundary t of the group starts tile
// mtile[g] + t and ends tile mtile[g] + t - 1.  The wave writes those tiles'
// records (absolute source offsets of every run, output offset, count), so a
// merge tile reads everything it needs with independent loads.
// Two phases: COARSE handles every COARSE_EVERY-th boundary (and the last)
// from the whole runs; FINE handles the others, starting from the windows
// between the cuts of the two coarse boundaries around them (the split of
// the first a elements only moves forward as a grows).
constexpr u32 COARSE_EVERY = 16;

template <typename K, int F, int M, bool FINE>
__global__ __launch_bounds__(256) void k_partition(Plan p, Level L, const K* __restrict__ src) {
  const u32 q = (blockIdx.x * blockDim.x + threadIdx.x) >> 6;
  const u32 lane = threadIdx.x & 63;
  const u32 total_tiles = p.mtile[L.NG];
  if (q >= total_tiles + L.NG) return;
  const u32 g = p.slot_grp[q];
  const u32 t0 = p.mtile[g];
  const u32 t = q - (t0 + g);
  const u32 nt = p.mtile[g + 1] - t0;
  if (t > nt || nt == 0) return;
  const bool coarse = (t % COARSE_EVERY) == 0 || t == nt;
  if (coarse == FINE) return;
  const u64 goff = p.grp_out[2 * (u64)g], glen = p.grp_out[2 * (u64)g + 1];
  const u64 roff = p.grp_run[((u64)g * F + lane % F) * 2];
  const u64 rlen = p.grp_run[((u64)g * F + lane % F) * 2 + 1];
  const u64 a = (u64)t * p.TM < glen ? (u64)t * p.TM : glen;
  u64 cut;
  if (a == 0) {
    cut = 0;
  } else if (a == glen) {
    cut = rlen;
  } else {
    u64 lo, hi;
    if (FINE) {
      const u32 tl = t - t % COARSE_EVERY;
      const u32 tr = tl + COARSE_EVERY < nt ? tl + COARSE_EVERY : nt;
      lo = p.rec_start[(u64)(t0 + tl) * F + lane % F] - roff;
      hi = p.rec_end[(u64)(t0 + tr - 1) * F + lane % F] - roff;
      if (hi > rlen) hi = rlen;
      if (lo > hi) lo = hi;
    } else {
      lo = a + rlen > glen ? a + rlen - glen : 0;
      hi = a < rlen ? a : rlen;
    }
    cut = wave_select<K, F, M>(src, roff, lo, hi, a, p.counters);
  }
  if (lane < (u32)F) {
    if (t < nt) p.rec_start[(u64)(t0 + t) * F + lane] = roff + cut;
    if (t > 0) p.rec_end[(u64)(t0 + t - 1) * F + lane] = roff + cut;
  }
  if (lane == 0 && t < nt) {
    p.rec_out[t0 + t] = goff + a;
    const u64 left = glen - a;
    p.rec_n[t0 + t] = (u32)(left < (u64)p.TM ? left : (u64)p.TM);
  }
}

// ----------------------------------------------------------------- merge tile
// LDS layout of the merge: element q lives at slot q + q / 8.  A thread merges
// IT = 8 consecutive outputs, so without the pad slot the 64 lanes of a wave
// would touch LDS at a stride of 8 elements and pile onto the same banks.
__device__ inline u32 pad8(u32 q) { return q + (q >> 3); }

// One thread's IT consecutive outputs [q0, q0 + IT) of a merge level where
// lists of `w` segments are merged pairwise (A = [a0, a1), B = [a1, b1), ties to
// A).  The outputs are produced into registers.  Only the first output needs
// a merge-path search: a thread whose range runs past the end of its pair
// goes on with the next pair, whose first output is that pair's start with
// nothing taken from either side yet.
template <typename K, bool IDX, int IT, int F>
__device__ inline void merge_thread(const K* ck, const uint16_t* ci, const u32* so, u32 w, u32 q0, u32 n,
                                    K (&ok)[IT], uint16_t (&oi)[IT]) {
  if (q0 >= n) return;
  // the pair holding output q0: the last pair start so[2wj] <= q0 (a binary
  // search over the F / 2w pair starts)
  u32 j = 0;
  for (u32 st = F / (4 * w); st >= 1; st >>= 1)
    if (so[2 * w * (j + st)] <= q0) j += st;
  const u32 a0 = so[2 * j * w];
  u32 a1 = so[min((2 * j + 1) * w, (u32)F)];
  u32 b1 = so[min((2 * j + 2) * w, (u32)F)];
  u32 ia, ib;
  {
    const u32 la = a1 - a0, lb = b1 - a1, diag = q0 - a0;
    u32 lo = diag > lb ? diag - lb : 0, hi = diag < la ? diag : la;
    while (lo < hi) {
      const u32 mid = (lo + hi) >> 1;
      if (ck[pad8(a0 + mid)] <= ck[pad8(a1 + diag - 1 - mid)]) lo = mid + 1; else hi = mid;
    }
    ia = a0 + lo;
    ib = a1 + diag - lo;
  }
  K ka = ia < a1 ? ck[pad8(ia)] : (K)0;
  K kb = ib < b1 ? ck[pad8(ib)] : (K)0;
#pragma unroll
  for (int i = 0; i < IT; ++i) {
    const u32 q = q0 + i;
    if (q < n) {
      // past the end of the pair (possibly several empty ones): the next
      // pair; it ends at so[F] = n > q at the latest
      while (q == b1) {
        ++j;
        ia = b1;
        a1 = so[min((2 * j + 1) * w, (u32)F)];
        b1 = so[min((2 * j + 2) * w, (u32)F)];
        ib = a1;
        ka = ia < a1 ? ck[pad8(ia)] : (K)0;
        kb = ib < b1 ? ck[pad8(ib)] : (K)0;
      }
      // branch-free step: emit the smaller front, reload only the side consumed
      const bool takeA = ib >= b1 || (ia < a1 && ka <= kb);
      const u32 from = takeA ? ia : ib;
      ok[i] = takeA ? ka : kb;
      if (IDX) oi[i] = ci[pad8(from)];
      ia += takeA ? 1u : 0u;
      ib += takeA ? 0u : 1u;
      // the element after the consumed one; past the end of its segment it is
      // never compared (the take test checks ia < a1 and ib < b1), and the
      // array has slack slots so that the read stays inside it
      const K nv = ck[pad8(from + 1)];
      ka = takeA ? nv : ka;
      kb = takeA ? kb : nv;
    }
  }
}

template <typename K, bool HASV, int F, int TM, int NT = 256>
__global__ __launch_bounds__(NT) void k_merge(Plan p, Level L, const K* __restrict__ src,
                                              const u32* __restrict__ srcv, K* __restrict__ dst,
                                              u32* __restrict__ dstv) {
  constexpr int IT = TM / NT, TP = TM + TM / 8 + 8;  // 8 slack slots past pad8(TM - 1)
  __shared__ K s_k[TP];
  __shared__ uint16_t s_i[HASV ? TP : 1];
  __shared__ u32 s_v[HASV ? TM : 1];
  __shared__ u64 s_roff[F];
  __shared__ u32 s_so[F + 1];
  const u32 tid = threadIdx.x;
  const u32 tile = blockIdx.x;
  if (tile >= p.mtile[L.NG]) return;
  // Segment r of this tile is source elements [rec_start[r], rec_end[r]); the
  // lengths are clamped so that a wrong record could never address memory
  // outside the tile's LDS or the run.
  if (tid < (u32)F) {
    const u64 a = p.rec_start[(u64)tile * F + tid], e = p.rec_end[(u64)tile * F + tid];
    s_roff[tid] = a;
    s_so[tid + 1] = (u32)(e > a ? (e - a < (u64)TM ? e - a : (u64)TM) : 0);
  }
  __syncthreads();
  if (tid == 0) {
    u32 acc = 0;
    const u32 cap = p.rec_n[tile] < (u32)TM ? p.rec_n[tile] : (u32)TM;
    s_so[0] = 0;
    for (int r = 1; r <= F; ++r) {
      acc += s_so[r];
      s_so[r] = acc < cap ? acc : cap;
    }
    // a tile can never hold more than its records allow; if it did, the
    // clamp above would drop elements: report it
    if (acc > cap) set_error(p.counters, E_SELECT);
  }
  __syncthreads();
  const u32 n = s_so[F];
  {
    // source positions first, then every load at once (past n: element 0,
    // always present when a tile exists), then the LDS stores; the run of
    // each element is the last run start <= its slot (a binary search over
    // the F starts, the IT searches interleaved)
    u64 e[IT];
    u32 r[IT];
#pragma unroll
    for (int i = 0; i < IT; ++i) r[i] = 0;
#pragma unroll
    for (int st = F / 2; st >= 1; st >>= 1) {
#pragma unroll
      for (int i = 0; i < IT; ++i) {
        const u32 q = tid + (u32)i * NT;
        if (s_so[r[i] + st] <= q) r[i] += st;
      }
    }
#pragma unroll
    for (int i = 0; i < IT; ++i) {
      const u32 q = tid + (u32)i * NT;
      e[i] = q < n ? s_roff[r[i]] + (q - s_so[r[i]]) : 0;
    }
    K kv[IT];
    u32 vv[HASV ? IT : 1];
#pragma unroll
    for (int i = 0; i < IT; ++i) {
      kv[i] = src[e[i]];
      if (HASV) vv[i] = srcv[e[i]];
    }
#pragma unroll
    for (int i = 0; i < IT; ++i) {
      const u32 q = tid + (u32)i * NT;
      if (q < n) {
        s_k[pad8(q)] = kv[i];
        if (HASV) {
          s_i[pad8(q)] = (uint16_t)q;
          s_v[q] = vv[i];
        }
      }
    }
  }
  __syncthreads();
  const u32 q0 = tid * IT;
  // up to four levels unrolled; a 32- or 64-way tile runs one copy of the
  // level's code (the levels differ in w only), so that the kernel stays
  // small in the instruction cache
#pragma unroll(F <= 16 ? 4 : 1)
  for (u32 w = 1; w < (u32)F; w <<= 1) {
    K ok[IT];
    uint16_t oi[IT];
    merge_thread<K, HASV, IT, F>(s_k, s_i, s_so, w, q0, n, ok, oi);
    __syncthreads();
    // q0 is a multiple of IT (4, 8 or 16) and (q0 mod 8) + i < 8 whenever
    // i < 8, so pad8(q0 + i) = pad8(q0) + i + i / 8
    static_assert(IT == 4 || IT == 8 || IT == 16, "outputs per thread");
    const u32 pq = pad8(q0);
#pragma unroll
    for (int i = 0; i < IT; ++i) {
      if (q0 + i < n) {
        s_k[pq + i + (i >> 3)] = ok[i];
        if (HASV) s_i[pq + i + (i >> 3)] = oi[i];
      }
    }
    __syncthreads();
  }
  const u64 out = p.rec_out[tile];
  if ((p.ky_top | p.ky_fm) == 0) {
    for (u32 q = tid; q < n; q += NT) {
      dst[out + q] = s_k[pad8(q)];
      if (HASV) dstv[out + q] = s_v[s_i[pad8(q)]];
    }
  } else {
    // the last pass of a signed or floating-point sort maps keys back
    for (u32 q = tid; q < n; q += NT) {
      dst[out + q] = key_out<K>(s_k[pad8(q)], p.ky_top, p.ky_fm);
      if (HASV) dstv[out + q] = s_v[s_i[pad8(q)]];
    }
  }
}

// ----------------------------------------------------------------- launchers
template <typename K, bool HASV, int F, int TM>
static void run_level(const Plan& p, const Level& L, const K* src, const u32* srcv, K* dst, u32* dstv,
                      u64 max_tiles, hipStream_t s) {
  // Fewest pivots that still give every run one per round: each round's
  // pivots cost a binary search in every run, and with one wave per boundary
  // the extra rounds are hidden by the many boundaries in flight.
  constexpr int M = F * F / 64 > 1 ? F * F / 64 : 1;
  { const int pe_ = prof_begin(s); hipLaunchKernelGGL(k_merge_plan, dim3(1), dim3(1024), 0, s, p, L); prof_end(pe_, "merge_plan", s); }
  const u64 slots = max_tiles + L.NG + 1;
  { const int pe_ = prof_begin(s); hipLaunchKernelGGL(k_slot_grp, dim3((u32)((slots + 255) / 256)), dim3(256), 0, s, p, L, (u32)slots); prof_end(pe_, "slot_grp", s); }
  { const int pe_ = prof_begin(s); hipLaunchKernelGGL((k_partition<K, F, M, false>), dim3((u32)((slots + 3) / 4)), dim3(256), 0, s, p, L, src); prof_end(pe_, "partition_coarse", s); }
  { const int pe_ = prof_begin(s); hipLaunchKernelGGL((k_partition<K, F, M, true>), dim3((u32)((slots + 3) / 4)), dim3(256), 0, s, p, L, src); prof_end(pe_, "partition_fine", s); }
  // eight outputs per thread for tiles of 2048 and 4096, four for 1024
  constexpr int NT = TM >= 2048 ? TM / 8 : 256;
  { const int pe_ = prof_begin(s); hipLaunchKernelGGL((k_merge<K, HASV, F, TM, NT>), dim3((u32)max_tiles), dim3(NT), 0, s, p, L, src, srcv, dst,
                     dstv); prof_end(pe_, "merge", s); }
}

template <typename K, bool HASV, int F>
static void run_level_tm(const Plan& p, const Level& L, const K* src, const u32* srcv, K* dst, u32* dstv,
                         u64 max_tiles, hipStream_t s) {
  switch (p.TM) {
    case 1024: run_level<K, HASV, F, 1024>(p, L, src, srcv, dst, dstv, max_tiles, s); break;
    case 4096: run_level<K, HASV, F, 4096>(p, L, src, srcv, dst, dstv, max_tiles, s); break;
    default: run_level<K, HASV, F, 2048>(p, L, src, srcv, dst, dstv, max_tiles, s); break;
  }
}

// One handler pass.  max_tiles bounds the pass's tile count (total_n/TM + groups).
template <typename K, bool HASV>
void launch_merge_level(const Plan& p, u32 level, const K* src, const u32* srcv, K* dst, u32* dstv,
                        hipStream_t s) {
  Level L;
  L.level = level;
  L.RS = 1;
  for (u32 x = 0; x < level; ++x) L.RS *= p.F;
  L.GS = L.RS * p.F;
  L.Q = (p.P + L.GS - 1) / L.GS;
  L.NG = p.B * p.P * L.Q;
  const u64 max_tiles = p.total_n / p.TM + L.NG;
  if (max_tiles == 0) return;
  switch (p.F) {
    case 2: run_level_tm<K, HASV, 2>(p, L, src, srcv, dst, dstv, max_tiles, s); break;
    case 4: run_level_tm<K, HASV, 4>(p, L, src, srcv, dst, dstv, max_tiles, s); break;
    case 16: run_level_tm<K, HASV, 16>(p, L, src, srcv, dst, dstv, max_tiles, s); break;
    default: run_level_tm<K, HASV, 8>(p, L, src, srcv, dst, dstv, max_tiles, s); break;
  }
}

// The one-pass handler's merge: tiles and their records come from the sampled
// tile bounds (k_samp_bounds); F = 32 or 64 runs per tile, TM = 2048 or 4096
// elements, eight per thread.
template <typename K, bool HASV>
void launch_merge_sampled(const Plan& p, u32 NG, u64 max_tiles, const K* src, const u32* srcv, K* dst, u32* dstv,
                          hipStream_t s) {
  Level L;
  L.level = 0;
  L.RS = 1;
  L.GS = p.F;
  L.Q = 1;
  L.NG = NG;
  if (max_tiles == 0) return;
  const int pe_ = prof_begin(s);
  const dim3 grid((u32)max_tiles);
  if (p.F == 32) {
    if (p.TM == 4096)
      hipLaunchKernelGGL((k_merge<K, HASV, 32, 4096, 512>), grid, dim3(512), 0, s, p, L, src, srcv, dst, dstv);
    else
      hipLaunchKernelGGL((k_merge<K, HASV, 32, 2048, 256>), grid, dim3(256), 0, s, p, L, src, srcv, dst, dstv);
  } else if (p.F == 64) {
    if (p.TM == 4096)
      hipLaunchKernelGGL((k_merge<K, HASV, 64, 4096, 512>), grid, dim3(512), 0, s, p, L, src, srcv, dst, dstv);
    else
      hipLaunchKernelGGL((k_merge<K, HASV, 64, 2048, 256>), grid, dim3(256), 0, s, p, L, src, srcv, dst, dstv);
  } else if (p.F == 16) {
    if (p.TM == 4096)
      hipLaunchKernelGGL((k_merge<K, HASV, 16, 4096, 512>), grid, dim3(512), 0, s, p, L, src, srcv, dst, dstv);
    else
      hipLaunchKernelGGL((k_merge<K, HASV, 16, 2048, 256>), grid, dim3(256), 0, s, p, L, src, srcv, dst, dstv);
  } else if (p.F == 8) {
    if (p.TM == 4096)
      hipLaunchKernelGGL((k_merge<K, HASV, 8, 4096, 512>), grid, dim3(512), 0, s, p, L, src, srcv, dst, dstv);
    else
      hipLaunchKernelGGL((k_merge<K, HASV, 8, 2048, 256>), grid, dim3(256), 0, s, p, L, src, srcv, dst, dstv);
  } else if (p.F == 4) {
    if (p.TM == 4096)
      hipLaunchKernelGGL((k_merge<K, HASV, 4, 4096, 512>), grid, dim3(512), 0, s, p, L, src, srcv, dst, dstv);
    else
      hipLaunchKernelGGL((k_merge<K, HASV, 4, 2048, 256>), grid, dim3(256), 0, s, p, L, src, srcv, dst, dstv);
  } else {
    if (p.TM == 4096)
      hipLaunchKernelGGL((k_merge<K, HASV, 2, 4096, 512>), grid, dim3(512), 0, s, p, L, src, srcv, dst, dstv);
    else
      hipLaunchKernelGGL((k_merge<K, HASV, 2, 2048, 256>), grid, dim3(256), 0, s, p, L, src, srcv, dst, dstv);
  }
  prof_end(pe_, "merge", s);
}

template void launch_merge_sampled<u32, false>(const Plan&, u32, u64, const u32*, const u32*, u32*, u32*, hipStream_t);
template void launch_merge_sampled<u32, true>(const Plan&, u32, u64, const u32*, const u32*, u32*, u32*, hipStream_t);
template void launch_merge_sampled<u64, false>(const Plan&, u32, u64, const u64*, const u32*, u64*, u32*, hipStream_t);
template void launch_merge_sampled<u64, true>(const Plan&, u32, u64, const u64*, const u32*, u64*, u32*, hipStream_t);

template void launch_merge_level<u32, false>(const Plan&, u32, const u32*, const u32*, u32*, u32*, hipStream_t);
template void launch_merge_level<u32, true>(const Plan&, u32, const u32*, const u32*, u32*, u32*, hipStream_t);
template void launch_merge_level<u64, false>(const Plan&, u32, const u64*, const u32*, u64*, u32*, hipStream_t);
template void launch_merge_level<u64, true>(const Plan&, u32, const u64*, const u32*, u64*, u32*, hipStream_t);

}  // namespace lbs
