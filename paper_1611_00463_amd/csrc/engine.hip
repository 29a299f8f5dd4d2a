// Host side of lbsort: argument checks, the workspace layout, and the launch
// sequence of one call (steps 1-6 of Section IV), all enqueued on the
// caller's stream with no host synchronisation in between.
#include <stdarg.h>
#include <stdlib.h>
#include <stdio.h>
#include <string.h>

#include <mutex>
#include <string>

#include "../../include/lbsort.h"
#include "lbsort_internal.hpp"
#include "tuning.hpp"

namespace lbs {

void launch_plan(const Plan& p, hipStream_t s);
void launch_fill_set(const FillSet& f, hipStream_t s);
template <typename K>
void launch_hist(const Plan& p, const K* src, hipStream_t s, u32 dlo = 0);
template <typename K, bool HASV>
void launch_small_sort(const Plan& p, const K* src, const u32* srcv, K* dst, u32* dstv, hipStream_t s);
template <typename K, bool HASV>
void launch_presorted(const Plan& p, const K* src, const u32* srcv, K* dst, u32* dstv, hipStream_t s);
template <typename K, bool HASV>
void launch_onesweep(const Plan& p, const K* src, const u32* srcv, K* dst, u32* dstv, u32 pass, hipStream_t s);
template <bool HASV>
void launch_group_fix(const Plan& p, const u64* src, const u32* srcv, u64* dst, u32* dstv, hipStream_t s);
template <bool HASV>
void launch_group_fix_mid(const Plan& p, const u64* src, const u32* srcv, u64* dst, u32* dstv, hipStream_t s);
template <bool HASV>
void launch_group_mid(const Plan& p, const u64* src, const u32* srcv, u64* dst, u32* dstv, u32 wgs, hipStream_t s);
template <typename K>
void launch_split(const Plan& p, const K* sorted, u64 max_samples, const void* out_offsets, void* out_counts,
                  void* out_send, void* out_cuts, void* out_split, hipStream_t s);
template <typename K, bool HASV>
void launch_merge_level(const Plan& p, u32 level, const K* src, const u32* srcv, K* dst, u32* dstv, hipStream_t s);
template <typename K, bool HASV>
void launch_handler_sampled(const Plan& p, const Plan& ps, const SampPlan& sp, u64 max_tiles, const K* sorted,
                            const u32* sortedv, K* dst, u32* dstv, hipStream_t s);
template <typename K>
void launch_key_out(K* a, u64 n, u64 top, u64 fm, hipStream_t s);
template <typename K>
void launch_search(const K* a, u64 n, const K* q, u64 nq, bool upper, u64 top, u64 fm, const u64* G, u32 P,
                   u64* pos, u32* part, hipStream_t s);
void launch_provenance(const u32* idx, u64 count, u64 n, u32 P, u32* blk, u32* off, hipStream_t s);
template <typename K>
void launch_search_index_build(const K* a, u64 n, void* index, hipStream_t s);
template <typename K>
void launch_search_indexed(const K* a, u64 n, const void* index, const K* q, u64 nq, bool upper, u64 top, u64 fm,
                           const u64* G, u32 P, u64* pos, u32* part, hipStream_t s);

static thread_local std::string g_last_error;

static int fail(int code, const char* fmt, ...) __attribute__((format(printf, 2, 3)));
static int fail(int code, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_last_error = buf;
  return code;
}

__global__ void k_seg2(u64* seg, u64 n) {
  if (threadIdx.x == 0) {
    seg[0] = 0;
    seg[1] = n;
  }
}

static inline u64 align256(u64 x) { return (x + 255) & ~(u64)255; }

// Key types: width in bytes (0 for an unknown type) and the masks of the
// order-preserving map onto unsigned integers (key_in in the kernels):
// signed integers flip the sign bit, IEEE floats flip the sign bit of
// non-negative numbers and every bit of negative ones (totalOrder).
static u32 key_width(int t) {
  switch (t) {
    case LBSORT_U32: case LBSORT_I32: case LBSORT_F32: return 4;
    case LBSORT_U64: case LBSORT_I64: case LBSORT_F64: return 8;
    default: return 0;
  }
}
static void key_masks(int t, u64& top, u64& fm) {
  const u32 w = key_width(t);
  const u64 sign = w == 8 ? (1ull << 63) : (1ull << 31);
  top = fm = 0;
  if (t == LBSORT_I32 || t == LBSORT_I64) top = sign;
  if (t == LBSORT_F32 || t == LBSORT_F64) {
    top = sign;
    fm = sign - 1;
  }
}

// Compute units of the current device (cached per device).
// The local sort of 64-bit keys: top three digits plus the group fix-up
// (default), or all eight radix passes when LBSORT_LOCAL_SORT=lsd.
static bool hybrid_local_sort() {
  const char* v = getenv("LBSORT_LOCAL_SORT");
  return !(v && strcmp(v, "lsd") == 0);
}

static u32 device_cus() {
  static int cached_dev = -1;
  static u32 cached = 0;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return 256;
  if (dev != cached_dev) {
    int cus = 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus <= 0) cus = 256;
    cached = (u32)cus;
    cached_dev = dev;
  }
  return cached;
}

struct Shape {
  int key_type, val_type;
  u32 B, P, s, inv, F, TM, L, D, rtile;
  u64 total_n;
  bool single;      // one instance whose size the host knows
  bool has_small, has_large;
  u64 max_tiles, max_samples;
  u32 ng0;          // merge groups of pass 0 (the largest pass)
  u64 mtiles;       // merge tiles of one pass, worst case
  bool local_only;  // step 1 only
  u32 handler;      // LBSORT_HANDLER_PASSES or LBSORT_HANDLER_ONE_PASS
  u32 presort;      // LBSORT_PRESORTED_DETECT or LBSORT_PRESORTED_IGNORE
  // one-pass handler: the sample problem (sample slots with gaps between
  // instances, its multi-pass merge: fan-in, tile, passes, groups, tiles)
  u64 s_max;
  u32 s_F, s_TM, s_L, s_ng0;
  u64 s_mtiles;
  u32 q;            // sorted samples per merge tile
};

struct Layout {
  u64 counters, blk_start, tstart, small_list, large_list, rem_prefix, tdesc, gflags, gflags2, presorted, midlist, samp_start, hist, status, samples, pool, lo, hi, cuts, Dm, G,
      splitters, mtile, rec_start, rec_end, rec_out, rec_n, slot_grp, grp_run, grp_out, tmpk, tmpv, seg, total;
  // one-pass handler
  u64 sseg, sbs, scuts, sDm, gsbase, ntile, skeys[2], svals[2], s_mtile, s_rec_start, s_rec_end, s_rec_out, s_rec_n,
      s_slot_grp, s_grp_run, s_grp_out, bsamp;
  bool bsamp_on;
};

// Entries of the mid-size group list: groups of more than GF_HALO keys in the
// large blocks of 64-bit keys.
static u64 mid_cap(const Shape& sh) {
  return key_width(sh.key_type) == 8 && sh.has_large ? sh.total_n / (GF_HALO + 1) + 1 : 0;
}

static Layout make_layout(const Shape& sh) {
  Layout l;
  const u64 K = key_width(sh.key_type);
  const u64 NB = (u64)sh.B * sh.P, P = sh.P, B = sh.B;
  u64 o = 0;
  auto take = [&](u64 bytes) {
    u64 at = o;
    o = align256(o + (bytes ? bytes : 1));
    return at;
  };
  l.counters = take(C_COUNT * 4);
  l.blk_start = take((NB + 1) * 8);
  l.tstart = take((NB + 1) * 4);
  l.small_list = take(NB * 4);
  l.large_list = take(NB * 4);
  l.rem_prefix = take((NB + 1) * 4);
  l.samp_start = take((NB + 1) * 8);
  l.hist = take(NB * sh.D * RADIX * 4);
  l.status = take(sh.max_tiles * RADIX * 8);
  l.tdesc = take(sh.max_tiles * sizeof(TileDesc));
  l.gflags = take(NB * 4);
  l.gflags2 = take(NB * 4);
  l.presorted = take(NB * 4);
  l.midlist = take(mid_cap(sh) * 8);
  l.samples = take(sh.max_samples * K);
  l.pool = take(sh.max_samples * K);
  l.lo = take(B * P * (P - 1) * 8);
  l.hi = take(B * P * (P - 1) * 8);
  l.cuts = take(B * P * (P + 1) * 8);
  l.Dm = take(B * (P + 1) * P * 8);
  l.G = take(B * (P + 1) * 8);
  l.splitters = take(B * (P - 1) * K);
  l.mtile = take(((u64)sh.ng0 + 1) * 4);
  l.rec_start = take(sh.mtiles * sh.F * 8);
  l.rec_end = take(sh.mtiles * sh.F * 8);
  l.rec_out = take(sh.mtiles * 8);
  l.rec_n = take(sh.mtiles * 4);
  l.slot_grp = take((sh.mtiles + sh.ng0 + 1) * 4);
  l.grp_run = take((u64)sh.ng0 * sh.F * 16);
  l.grp_out = take((u64)sh.ng0 * 16);
  const u64 stages = (u64)sh.D + sh.L;
  const bool need_tmp = stages > 1;
  l.tmpk = take(need_tmp ? sh.total_n * K : 0);
  l.tmpv = take(need_tmp && sh.val_type ? sh.total_n * 4 : 0);
  l.seg = take(16);
  const bool one = sh.handler == LBSORT_HANDLER_ONE_PASS && sh.L > 0;
  const u64 sm = one ? sh.s_max : 0;
  l.sseg = take(one ? (B + 1) * 8 : 0);
  l.sbs = take(one ? (NB + 1) * 8 : 0);
  l.scuts = take(one ? B * P * (P + 1) * 8 : 0);
  l.sDm = take(one ? B * (P + 1) * P * 8 : 0);
  l.gsbase = take(one ? NB * 8 : 0);
  l.ntile = take(one ? NB * 4 : 0);
  for (int x = 0; x < 2; ++x) {
    l.skeys[x] = take(sm * K);
    l.svals[x] = take(sm * 4);
  }
  l.s_mtile = take(one ? ((u64)sh.s_ng0 + 1) * 4 : 0);
  l.s_rec_start = take(one ? sh.s_mtiles * sh.s_F * 8 : 0);
  l.s_rec_end = take(one ? sh.s_mtiles * sh.s_F * 8 : 0);
  l.s_rec_out = take(one ? sh.s_mtiles * 8 : 0);
  l.s_rec_n = take(one ? sh.s_mtiles * 4 : 0);
  l.s_slot_grp = take(one ? (sh.s_mtiles + sh.s_ng0 + 1) * 4 : 0);
  l.s_grp_run = take(one ? (u64)sh.s_ng0 * sh.s_F * 16 : 0);
  l.s_grp_out = take(one ? (u64)sh.s_ng0 * 16 : 0);
  // block samples: ceil(n_i / m) keys of block i at floor(start_i / m) + i
  l.bsamp_on = one && K == 8 && hybrid_local_sort();
  l.bsamp = take(l.bsamp_on ? (sh.total_n / SAMP_STRIDE + NB + 1) * K : 0);
  l.total = o;
  return l;
}

static int make_shape(int key_type, int val_type, u32 B, u64 total_n, const lbsort_params* prm, bool local_only,
                      Shape& sh) {
  if (!key_width(key_type))
    return fail(LBSORT_ERR_INVALID_ARG, "key_type must be one of LBSORT_U32..LBSORT_F64 (got %d)", key_type);
  if (val_type != LBSORT_NOVAL && val_type != LBSORT_VAL_U32 && val_type != LBSORT_VAL_INDEX)
    return fail(LBSORT_ERR_INVALID_ARG, "val_type must be LBSORT_NOVAL, LBSORT_VAL_U32 or LBSORT_VAL_INDEX (got %d)",
                val_type);
  if (val_type == LBSORT_VAL_INDEX && B == 1 && total_n > (1ull << 32))
    return fail(LBSORT_ERR_UNSUPPORTED, "LBSORT_VAL_INDEX needs n <= 2^32 (32-bit positions)");
  lbsort_params d = {1, 0, LBSORT_INV_COUNT, 0, 0, 0, 0, 0, 0};
  const lbsort_params& p = prm ? *prm : d;
  if (p.P < 1 || p.P > LBSORT_MAX_P) return fail(LBSORT_ERR_INVALID_ARG, "P must be in [1, %d] (got %u)", LBSORT_MAX_P, p.P);
  if (p.investigator > 2) return fail(LBSORT_ERR_INVALID_ARG, "unknown investigator mode %u", p.investigator);
  if (p.s > LBSORT_MAX_SAMPLES) return fail(LBSORT_ERR_INVALID_ARG, "s must be <= %u (got %u)", LBSORT_MAX_SAMPLES, p.s);
  if (p.presorted > LBSORT_PRESORTED_IGNORE)
    return fail(LBSORT_ERR_INVALID_ARG, "presorted must be 0, LBSORT_PRESORTED_DETECT or LBSORT_PRESORTED_IGNORE (got %u)",
                p.presorted);
  if (p.handler > LBSORT_HANDLER_ONE_PASS)
    return fail(LBSORT_ERR_INVALID_ARG, "handler must be 0, LBSORT_HANDLER_PASSES or LBSORT_HANDLER_ONE_PASS (got %u)",
                p.handler);
  if (p.handler != LBSORT_HANDLER_ONE_PASS && p.fanin != 0 && p.fanin != 2 && p.fanin != 4 && p.fanin != 8 &&
      p.fanin != 16)
    return fail(LBSORT_ERR_INVALID_ARG, "fanin must be 0, 2, 4, 8 or 16 (got %u)", p.fanin);
  if (p.merge_tile != 0 && p.merge_tile != 1024 && p.merge_tile != 2048 && p.merge_tile != 4096)
    return fail(LBSORT_ERR_INVALID_ARG, "merge_tile must be 0, 1024, 2048 or 4096 (got %u)", p.merge_tile);
  if (p.radix_tile != 0 && p.radix_tile != RTILE_SMALL && p.radix_tile != RTILE_LARGE &&
      !(p.radix_tile == RTILE_HUGE && key_width(key_type) == 4))
    return fail(LBSORT_ERR_INVALID_ARG, "radix_tile must be 0, %u, %u or (32-bit keys) %u (got %u)", RTILE_SMALL,
                RTILE_LARGE, RTILE_HUGE, p.radix_tile);
  if (p.reserved != 0) return fail(LBSORT_ERR_INVALID_ARG, "reserved must be 0");
  if (B < 1) return fail(LBSORT_ERR_INVALID_ARG, "B must be >= 1");
  if (total_n >= (1ull << 44)) return fail(LBSORT_ERR_UNSUPPORTED, "total_n must be < 2^44");
  if ((u64)B * p.P > (1ull << 26)) return fail(LBSORT_ERR_UNSUPPORTED, "B * P must be <= 2^26");
  sh.key_type = key_type;
  sh.val_type = val_type;
  sh.B = B;
  sh.P = p.P;
  sh.total_n = total_n;
  sh.inv = p.investigator;
  sh.local_only = local_only;
  const u32 kb = key_width(key_type);
  sh.D = kb * 8 / RADIX_BITS;
  // default budget: the largest multiple of P samples within one 256 KB read
  // buffer over all processors (that budget itself when it is below P)
  const u32 budget = 262144u / (p.P * kb);
  sh.s = p.s ? p.s : (budget >= p.P ? budget / p.P * p.P : (budget > 0 ? budget : 1u));
  // merge fan-in and tile: explicit, else tuned, else defaults
  // tuned settings depend on the widths only
  Tuned tu = tuning_lookup(kb, val_type != LBSORT_NOVAL, total_n / B, B, p.P);
  // step 6: one pass with sampled tiles (P <= 64, positions in 32 bits), or
  // F-way passes with exact tiles
  const bool one_ok = p.P >= 2 && p.P <= 64 && total_n <= (1ull << 32);
  u32 handler = p.handler;
  // an explicit fan-in of the passes, or a tile only they take, implies them
  if (!handler && ((p.fanin && p.fanin <= 16) || p.merge_tile == 1024)) handler = LBSORT_HANDLER_PASSES;
  if (!handler) handler = tu.handler;
  // untuned: the exact passes (the one-pass schedule wins on inputs with
  // heavy duplicates, where exact selection needs many rounds; the tuner
  // picks it there)
  if (!handler) handler = LBSORT_HANDLER_PASSES;
  if (handler == LBSORT_HANDLER_ONE_PASS && !one_ok) {
    if (p.handler == LBSORT_HANDLER_ONE_PASS && p.P >= 2)
      return fail(LBSORT_ERR_UNSUPPORTED, "the one-pass handler needs P <= 64 and total_n <= 2^32");
    handler = LBSORT_HANDLER_PASSES;
  }
  if (p.P < 2) handler = LBSORT_HANDLER_PASSES;
  sh.handler = handler;
  u32 pow2P = 2;
  while (pow2P < p.P) pow2P *= 2;
  u32 F;
  if (handler == LBSORT_HANDLER_ONE_PASS) {
    if (p.fanin && p.fanin != pow2P)
      return fail(LBSORT_ERR_INVALID_ARG, "with the one-pass handler fanin must be 0 or %u for P = %u (got %u)", pow2P,
                  p.P, p.fanin);
    F = pow2P;
    if (p.merge_tile == 1024)
      return fail(LBSORT_ERR_INVALID_ARG, "the one-pass handler's merge_tile must be 2048 or 4096");
    sh.TM = p.merge_tile ? p.merge_tile : (tu.merge_tile >= 2048 && tu.handler == handler ? tu.merge_tile : 4096u);
    if (sh.TM / SAMP_STRIDE <= p.P) sh.TM = 4096;
  } else {
    F = p.fanin ? p.fanin : (tu.handler == handler ? tu.fanin : 0);
    if (!F) {
      F = pow2P < 16 ? pow2P : 16;
      if (p.P > 16) F = 8;
    }
    sh.TM = p.merge_tile ? p.merge_tile : (tu.merge_tile && tu.handler == handler ? tu.merge_tile : 2048u);
  }
  sh.F = F;
  sh.rtile = p.radix_tile ? p.radix_tile : (tu.radix_tile ? tu.radix_tile : RTILE_LARGE);
  sh.presort = p.presorted ? p.presorted : (tu.presorted ? tu.presorted : LBSORT_PRESORTED_DETECT);
  if (sh.rtile == RTILE_HUGE && kb != 4) sh.rtile = RTILE_LARGE;  // a tuned entry of another key width
  u32 L = 0;
  for (u64 span = 1; span < p.P; span *= F) ++L;
  sh.L = local_only ? 0 : L;
  const u64 NB = (u64)B * p.P;
  sh.single = (B == 1);
  if (sh.single) {
    sh.has_small = sh.has_large = false;
    sh.max_tiles = 0;
    sh.max_samples = 0;
    for (u32 i = 0; i < p.P; ++i) {
      const u64 n = (u64)(((unsigned __int128)(i + 1) * total_n) / p.P) - (u64)(((unsigned __int128)i * total_n) / p.P);
      if (n >= (1ull << 32)) return fail(LBSORT_ERR_UNSUPPORTED, "a block of 2^32 keys or more (raise P)");
      if (n > (u64)SMALL_TILE) {
        sh.has_large = true;
        sh.max_tiles += (n + sh.rtile - 1) / sh.rtile;
      } else if (n > 0) {
        sh.has_small = true;
      }
      sh.max_samples += n < sh.s ? n : sh.s;
    }
  } else {
    sh.has_small = sh.has_large = true;
    sh.max_tiles = total_n / sh.rtile + NB;
    const u64 cap = NB * sh.s;
    sh.max_samples = total_n < cap ? total_n : cap;
  }
  if (sh.max_tiles >= (1ull << 31)) return fail(LBSORT_ERR_UNSUPPORTED, "too many radix tiles");
  const u64 Q0 = (p.P + F - 1) / F;
  sh.ng0 = (u32)(NB * Q0);
  sh.mtiles = sh.L ? total_n / sh.TM + sh.ng0 + 1 : 0;
  sh.s_max = 0;
  sh.s_F = sh.s_TM = sh.s_L = sh.s_ng0 = sh.q = 0;
  sh.s_mtiles = 0;
  if (sh.handler == LBSORT_HANDLER_ONE_PASS && sh.L > 0) {
    // every run (B P^2 of them) adds at most two samples above len / m
    // (its first element, and the block positions that are multiples of m)
    const u64 PP = (u64)p.P * p.P;
    sh.s_max = total_n / SAMP_STRIDE + (u64)B * (2 * PP + 1) + 1;
    sh.q = sh.TM / SAMP_STRIDE - p.P;
    sh.mtiles = (total_n / SAMP_STRIDE + 2 * B * PP) / sh.q + NB + 1;
    sh.s_F = pow2P < 16 ? pow2P : 16;
    if (p.P > 16) sh.s_F = 8;
    sh.s_TM = 2048;
    sh.s_L = 0;
    for (u64 span = 1; span < p.P; span *= sh.s_F) ++sh.s_L;
    sh.s_ng0 = (u32)(NB * ((p.P + sh.s_F - 1) / sh.s_F));
    sh.s_mtiles = sh.s_max / sh.s_TM + sh.s_ng0 + 1;
  }
  return LBSORT_OK;
}

template <typename K, bool HASV>
static int run(const Shape& sh, const Layout& lay, const K* kin, const u32* vin, K* kout, u32* vout,
               const u64* seg_in, const lbsort_parts* parts, char* ws, hipStream_t st) {
  Plan p;
  memset(&p, 0, sizeof p);
  p.gshift = sh.key_type == LBSORT_F64 ? 32u : 40u;
  p.B = sh.B;
  p.P = sh.P;
  p.NB = sh.B * sh.P;
  p.s = sh.s;
  p.D = sh.D;
  p.inv = sh.inv;
  p.F = sh.F;
  p.L = sh.L;
  p.TM = sh.TM;
  p.max_tiles = (u32)sh.max_tiles;
  p.rtile = sh.rtile;
  p.nq = NQ;
  p.persist_wgs = device_cus() * 4;
  p.total_n = sh.total_n;
  p.blk_start = (u64*)(ws + lay.blk_start);
  p.tstart = (u32*)(ws + lay.tstart);
  p.small_list = (u32*)(ws + lay.small_list);
  p.large_list = (u32*)(ws + lay.large_list);
  p.rem_prefix = (u32*)(ws + lay.rem_prefix);
  p.tdesc = (TileDesc*)(ws + lay.tdesc);
  p.gflags = (u32*)(ws + lay.gflags);
  p.gflags2 = (u32*)(ws + lay.gflags2);
  u32* const presorted = (u32*)(ws + lay.presorted);
  p.midlist = (u64*)(ws + lay.midlist);
  p.mid_cap = mid_cap(sh);
  p.counters = (u32*)(ws + lay.counters);
  p.hist = (u32*)(ws + lay.hist);
  p.status = (u64*)(ws + lay.status);
  p.samp_start = (u64*)(ws + lay.samp_start);
  p.samples = ws + lay.samples;
  p.pool = ws + lay.pool;
  p.lo = (u64*)(ws + lay.lo);
  p.hi = (u64*)(ws + lay.hi);
  p.cuts = (u64*)(ws + lay.cuts);
  p.Dm = (u64*)(ws + lay.Dm);
  p.G = (u64*)(ws + lay.G);
  p.splitters = ws + lay.splitters;
  p.mtile = (u32*)(ws + lay.mtile);
  p.rec_start = (u64*)(ws + lay.rec_start);
  p.rec_end = (u64*)(ws + lay.rec_end);
  p.rec_out = (u64*)(ws + lay.rec_out);
  p.rec_n = (u32*)(ws + lay.rec_n);
  p.slot_grp = (u32*)(ws + lay.slot_grp);
  p.grp_run = (u64*)(ws + lay.grp_run);
  p.grp_out = (u64*)(ws + lay.grp_out);
  p.ng_max = sh.ng0;
  p.mtiles_max = (u32)sh.mtiles;
  // block samples where the local sort's last writer is the group fix-up
  // (64-bit keys on the fix-up path), which writes blocks in position order
  if (lay.bsamp_on) p.bsamp = ws + lay.bsamp;
  p.vidx = sh.val_type == LBSORT_VAL_INDEX;
  if (seg_in) {
    p.seg = seg_in;
  } else {
    u64* seg = (u64*)(ws + lay.seg);
    hipLaunchKernelGGL(k_seg2, dim3(1), dim3(64), 0, st, seg, sh.total_n);
    p.seg = seg;
  }
  // launches that read keys_in map the keys (px); those that write keys_out
  // or the splitters map them back (py)
  u64 top, fm;
  key_masks(sh.key_type, top, fm);
  Plan px = p, py = p;
  px.kx_top = top;
  px.kx_fm = fm;
  py.ky_top = top;
  py.ky_fm = fm;
  K* tk = (K*)(ws + lay.tmpk);
  u32* tv = (u32*)(ws + lay.tmpv);
  const u32 S = sh.D + sh.L;
  auto dk = [&](u32 j) -> K* { return ((S - 1 - j) % 2 == 0) ? kout : tk; };
  auto dv = [&](u32 j) -> u32* { return ((S - 1 - j) % 2 == 0) ? vout : tv; };

  // the fix-up path of 64-bit keys needs the counts of the top digits only:
  // three, or four for doubles (their sign and exponent leave few distinct
  // values in the top 24 bits, so groups of equal top 24 bits run to
  // hundreds of keys; one more pass is cheaper than the mid-size group sort)
  const bool hybrid = sizeof(K) == 8 && hybrid_local_sort();
  const u32 ntop = (64u - p.gshift) / RADIX_BITS;
  {
    // every word that must start at a known value, in one launch
    FillSet f;
    f.add(p.counters, C_COUNT, 0);
    if (sh.has_large) {
      f.add(p.hist, (u64)p.NB * sh.D * RADIX, 0);
      f.add((u32*)p.status, sh.max_tiles * RADIX * 2, 0);
      if (sh.presort == LBSORT_PRESORTED_DETECT) f.add(presorted, p.NB, 3u);
      if (sizeof(K) == 8 && hybrid) {
        f.add(p.gflags, p.NB, 0);
        f.add(p.gflags2, p.NB, 0);
      }
    }
    launch_fill_set(f, st);
  }
  launch_plan(p, st);
  // the fix-up path's top-digit passes leave out a digit that no block needs
  Plan ph = px;
  ph.bsamp = nullptr;  // the top-digit passes do not write the local sort's output
  if (hybrid) {
    ph.run_slot = C_RUN_TOP;
    ph.run_mask = ntop == 4 ? 0xF0u : 0xE0u;  // digits 4 (doubles), 5, 6, 7
  }
  if (sh.has_large) {
    // the histogram also finds the large blocks that are already in order
    // (or in reverse order); those are written to the local sort's output
    // at once, and the radix passes are planned again without them
    const bool detect = sh.presort == LBSORT_PRESORTED_DETECT;
    Plan hp = hybrid ? ph : px;
    hp.presorted = detect ? presorted : nullptr;
    launch_hist<K>(hp, kin, st, hybrid ? 8u - ntop : 0u);
    if (detect) {
      Plan cp = px;
      cp.presorted = presorted;
      launch_presorted<K, HASV>(cp, kin, vin, dk(sh.D - 1), dv(sh.D - 1), st);
      Plan rp = p;
      rp.skip = presorted;
      launch_plan(rp, st);
    }
  }
  if (sh.has_small) launch_small_sort<K, HASV>(px, kin, vin, dk(sh.D - 1), dv(sh.D - 1), st);
  if (sh.has_large) {
    if constexpr (sizeof(K) == 8) {
      if (hybrid) {
        // 64-bit keys: the three highest digits first (four for doubles:
        // blocks grouped by key >> gshift), then the group fix-up into the
        // step-1 output F; the blocks it flags are sorted again over all eight
        // digits.
        K* const F = dk(sh.D - 1);
        u32* const FV = dv(sh.D - 1);
        K* const O = F == kout ? tk : kout;
        u32* const OV = HASV ? (FV == vout ? tv : vout) : nullptr;
        // the passes that run read the input first and leave their result in O
        ph.pass_out = O;
        ph.pass_outv = OV;
        ph.pass_tmp = F;
        ph.pass_tmpv = FV;
        for (u32 j = 8 - ntop; j < 8; ++j) launch_onesweep<K, HASV>(ph, kin, vin, O, OV, j, st);
        launch_group_fix<HASV>(p, (const u64*)O, OV, (u64*)F, FV, st);
        launch_group_fix_mid<HASV>(p, (const u64*)O, OV, (u64*)F, FV, st);
        launch_group_mid<HASV>(p, (const u64*)O, OV, (u64*)F, FV, device_cus() * 8, st);
        Plan q = p;
        q.only = p.gflags2;
        q.epoch_base = 8;  // the status words of the passes above stay valid for epochs 5..8
        {
          FillSet f;
          f.add(p.counters + C_TICKET, NQ * sh.D, 0);
          f.add(p.hist, (u64)p.NB * sh.D * RADIX, 0);
          launch_fill_set(f, st);
        }
        launch_plan(q, st);
        Plan qx = q;
        qx.kx_top = top;
        qx.kx_fm = fm;
        // only the digits that reorder some flagged block are passed over; the
        // first pass that runs reads the input (and maps typed keys), the
        // last writes F (the kernels pick their buffers from the digit mask)
        qx.run_slot = C_RUN_REDO;
        qx.run_mask = 0xFFu;
        qx.pass_out = F;
        qx.pass_outv = FV;
        qx.pass_tmp = O;
        qx.pass_tmpv = OV;
        launch_hist<K>(qx, kin, st);
        for (u32 j = 0; j < sh.D; ++j) launch_onesweep<K, HASV>(qx, kin, vin, F, FV, j, st);
      } else {
        for (u32 j = 0; j < sh.D; ++j)
          launch_onesweep<K, HASV>(j ? p : px, j ? dk(j - 1) : kin, j ? dv(j - 1) : vin, dk(j), dv(j), j, st);
      }
    } else {
      for (u32 j = 0; j < sh.D; ++j)
        launch_onesweep<K, HASV>(j ? p : px, j ? dk(j - 1) : kin, j ? dv(j - 1) : vin, dk(j), dv(j), j, st);
    }
  }
  if (!sh.local_only) {
    const K* sorted = dk(sh.D - 1);
    launch_split<K>(py, sorted, sh.max_samples, parts->part_offsets, parts->part_counts, parts->send_counts,
                    parts->cuts, parts->splitters, st);
    if (sh.handler == LBSORT_HANDLER_ONE_PASS && sh.L == 1) {
      // the sample problem: its own layout of blocks, cuts and range table,
      // and its own merge records (the main tile records are written later)
      SampPlan sp;
      sp.sseg = (u64*)(ws + lay.sseg);
      sp.sbs = (u64*)(ws + lay.sbs);
      sp.scuts = (u64*)(ws + lay.scuts);
      sp.sDm = (u64*)(ws + lay.sDm);
      sp.gsbase = (u64*)(ws + lay.gsbase);
      sp.ntile = (u32*)(ws + lay.ntile);
      for (int x = 0; x < 2; ++x) {
        sp.skeys[x] = ws + lay.skeys[x];
        sp.svals[x] = (u32*)(ws + lay.svals[x]);
      }
      sp.m = SAMP_STRIDE;
      sp.q = sh.q;
      Plan ps = p;
      ps.seg = sp.sseg;
      ps.blk_start = sp.sbs;
      ps.cuts = sp.scuts;
      ps.Dm = sp.sDm;
      ps.F = sh.s_F;
      ps.TM = sh.s_TM;
      ps.L = sh.s_L;
      ps.total_n = sh.s_max;
      ps.mtile = (u32*)(ws + lay.s_mtile);
      ps.rec_start = (u64*)(ws + lay.s_rec_start);
      ps.rec_end = (u64*)(ws + lay.s_rec_end);
      ps.rec_out = (u64*)(ws + lay.s_rec_out);
      ps.rec_n = (u32*)(ws + lay.s_rec_n);
      ps.slot_grp = (u32*)(ws + lay.s_slot_grp);
      ps.grp_run = (u64*)(ws + lay.s_grp_run);
      ps.grp_out = (u64*)(ws + lay.s_grp_out);
      ps.ng_max = sh.s_ng0;
      ps.mtiles_max = (u32)sh.s_mtiles;
      launch_handler_sampled<K, HASV>(py, ps, sp, sh.mtiles, sorted, dv(sh.D - 1), dk(sh.D), dv(sh.D), st);
    } else {
      for (u32 l = 0; l < sh.L; ++l)
        launch_merge_level<K, HASV>(l + 1 == sh.L ? py : p, l, dk(sh.D - 1 + l), dv(sh.D - 1 + l), dk(sh.D + l),
                                    dv(sh.D + l), st);
    }
  }
  // without a merge pass the local sort wrote keys_out: map it back in place
  if (sh.L == 0 && (top | fm) != 0) launch_key_out<K>(kout, sh.total_n, top, fm, st);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return fail(LBSORT_ERR_HIP, "kernel launch failed: %s", hipGetErrorString(e));
  return LBSORT_OK;
}

static int dispatch(const Shape& sh, const void* kin, const void* vin, void* kout, void* vout, const u64* seg,
                    const lbsort_parts* parts, void* ws, size_t* ws_bytes, void* stream) {
  const Layout lay = make_layout(sh);
  if (!ws_bytes) return fail(LBSORT_ERR_INVALID_ARG, "ws_bytes must not be NULL");
  if (!ws) {
    *ws_bytes = lay.total;
    return LBSORT_OK;
  }
  if (*ws_bytes < lay.total)
    return fail(LBSORT_ERR_WORKSPACE_TOO_SMALL, "workspace of %zu bytes, need %llu", *ws_bytes,
                (unsigned long long)lay.total);
  if (((uintptr_t)ws & 255) != 0) return fail(LBSORT_ERR_INVALID_ARG, "workspace must be 256-byte aligned");
  if (sh.total_n > 0 && (!kin || !kout)) return fail(LBSORT_ERR_INVALID_ARG, "keys_in/keys_out must not be NULL");
  if (sh.val_type == LBSORT_VAL_U32 && sh.total_n > 0 && (!vin || !vout))
    return fail(LBSORT_ERR_INVALID_ARG, "vals_in/vals_out must not be NULL with LBSORT_VAL_U32");
  if (sh.val_type == LBSORT_VAL_INDEX) {
    if (sh.total_n > 0 && !vout) return fail(LBSORT_ERR_INVALID_ARG, "vals_out must not be NULL with LBSORT_VAL_INDEX");
    vin = nullptr;  // the values are generated
  }
  if (!sh.local_only && (!parts || !parts->part_offsets))
    return fail(LBSORT_ERR_INVALID_ARG, "parts->part_offsets is required");
  hipStream_t st = (hipStream_t)stream;
  char* w = (char*)ws;
  const bool v = sh.val_type != LBSORT_NOVAL;
  if (key_width(sh.key_type) == 8) {
    if (v) return run<u64, true>(sh, lay, (const u64*)kin, (const u32*)vin, (u64*)kout, (u32*)vout, seg, parts, w, st);
    return run<u64, false>(sh, lay, (const u64*)kin, nullptr, (u64*)kout, nullptr, seg, parts, w, st);
  }
  if (v) return run<u32, true>(sh, lay, (const u32*)kin, (const u32*)vin, (u32*)kout, (u32*)vout, seg, parts, w, st);
  return run<u32, false>(sh, lay, (const u32*)kin, nullptr, (u32*)kout, nullptr, seg, parts, w, st);
}

// ----------------------------------------------------------------- static scratch
// Scratch of the allocation-free entry point: a file-scope device array
// (each device the library runs on holds its own copy until the process
// ends).  In host code `scratch` names a host-side stand-in, not device
// memory: its device address is taken once per device with
// hipGetSymbolAddress, and only that address is handed to kernels.
constexpr u64 NOALLOC_SCRATCH_BYTES = LBSORT_NOALLOC_SCRATCH_BYTES;
static __device__ __align__(256) unsigned char scratch[NOALLOC_SCRATCH_BYTES];

constexpr int MAX_DEVICES = 64;
static std::mutex g_scratch_mu;
static void* g_scratch_ptr[MAX_DEVICES];

// Device address of `scratch` on the current device (looked up on the first
// call made with that device current).
static int scratch_ptr(void** out) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return fail(LBSORT_ERR_HIP, "hipGetDevice failed: %s", hipGetErrorString(e));
  if (dev < 0 || dev >= MAX_DEVICES) return fail(LBSORT_ERR_UNSUPPORTED, "device %d beyond the %d supported", dev, MAX_DEVICES);
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* ptr = nullptr;
    e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr)
      return fail(LBSORT_ERR_HIP, "hipGetSymbolAddress(scratch) failed on device %d: %s", dev, hipGetErrorString(e));
    g_scratch_ptr[dev] = ptr;
  }
  *out = g_scratch_ptr[dev];
  return LBSORT_OK;
}

// The call's latched device error bits, copied out for the caller.
__global__ void k_copy_err(const u32* counters, u32* out) {
  if (threadIdx.x == 0) *out = counters[C_ERR];
}

}  // namespace lbs

using namespace lbs;

extern "C" {

int lbsort_sort_keys(int key_type, const void* keys_in, void* keys_out, uint64_t n, const lbsort_params* params,
                     const lbsort_parts* parts, void* ws, size_t* ws_bytes, void* stream) {
  Shape sh;
  int rc = make_shape(key_type, LBSORT_NOVAL, 1, n, params, false, sh);
  if (rc) return rc;
  return dispatch(sh, keys_in, nullptr, keys_out, nullptr, nullptr, parts, ws, ws_bytes, stream);
}

int lbsort_sort_pairs(int key_type, int val_type, const void* keys_in, const void* vals_in, void* keys_out,
                      void* vals_out, uint64_t n, const lbsort_params* params, const lbsort_parts* parts, void* ws,
                      size_t* ws_bytes, void* stream) {
  Shape sh;
  int rc = make_shape(key_type, val_type, 1, n, params, false, sh);
  if (rc) return rc;
  return dispatch(sh, keys_in, vals_in, keys_out, vals_out, nullptr, parts, ws, ws_bytes, stream);
}

int lbsort_sort_pairs_noalloc(int key_type, int val_type, const void* keys_in, const void* vals_in, void* keys_out,
                              void* vals_out, uint64_t n, const lbsort_params* params, const lbsort_parts* parts,
                              uint32_t* dev_err, void* stream) {
  Shape sh;
  int rc = make_shape(key_type, val_type, 1, n, params, false, sh);
  if (rc) return rc;
  const Layout lay = make_layout(sh);
  if (lay.total > NOALLOC_SCRATCH_BYTES)
    return fail(LBSORT_ERR_UNSUPPORTED,
                "n = %llu needs %llu bytes of scratch; the allocation-free entry point has %llu (use lbsort_sort_pairs "
                "with a workspace)",
                (unsigned long long)n, (unsigned long long)lay.total, (unsigned long long)NOALLOC_SCRATCH_BYTES);
  void* ws = nullptr;
  rc = scratch_ptr(&ws);
  if (rc) return rc;
  size_t have = (size_t)NOALLOC_SCRATCH_BYTES;
  rc = dispatch(sh, keys_in, vals_in, keys_out, vals_out, nullptr, parts, ws, &have, stream);
  if (rc) return rc;
  if (dev_err) {
    hipLaunchKernelGGL(k_copy_err, dim3(1), dim3(64), 0, (hipStream_t)stream, (const u32*)ws, dev_err);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return fail(LBSORT_ERR_HIP, "kernel launch failed: %s", hipGetErrorString(e));
  }
  return LBSORT_OK;
}

int lbsort_sort_batch(int key_type, int val_type, const void* keys_in, const void* vals_in, void* keys_out,
                      void* vals_out, const uint64_t* seg_offsets, uint32_t B, uint64_t total_n,
                      const lbsort_params* params, const lbsort_parts* parts, void* ws, size_t* ws_bytes,
                      void* stream) {
  Shape sh;
  int rc = make_shape(key_type, val_type, B, total_n, params, false, sh);
  if (rc) return rc;
  if (!seg_offsets) return fail(LBSORT_ERR_INVALID_ARG, "seg_offsets must not be NULL");
  return dispatch(sh, keys_in, vals_in, keys_out, vals_out, seg_offsets, parts, ws, ws_bytes, stream);
}

int lbsort_resolve_params(int key_type, int val_type, uint32_t B, uint64_t total_n, const lbsort_params* params,
                          lbsort_params* out) {
  if (!out) return fail(LBSORT_ERR_INVALID_ARG, "out must not be NULL");
  Shape sh;
  int rc = make_shape(key_type, val_type, B, total_n, params, false, sh);
  if (rc) return rc;
  lbsort_params r = {sh.P, sh.s, sh.inv, sh.F, sh.TM, sh.rtile, sh.handler, sh.presort, 0};
  *out = r;
  return LBSORT_OK;
}

int lbsort_local_sort(int key_type, int val_type, const void* keys_in, const void* vals_in, void* keys_out,
                      void* vals_out, const uint64_t* seg_offsets, uint32_t B, uint64_t total_n,
                      const lbsort_params* params, void* ws, size_t* ws_bytes, void* stream) {
  Shape sh;
  int rc = make_shape(key_type, val_type, B, total_n, params, true, sh);
  if (rc) return rc;
  if (!seg_offsets) return fail(LBSORT_ERR_INVALID_ARG, "seg_offsets must not be NULL");
  return dispatch(sh, keys_in, vals_in, keys_out, vals_out, seg_offsets, nullptr, ws, ws_bytes, stream);
}

int lbsort_search(int key_type, const void* sorted_keys, uint64_t n, const void* queries, uint64_t nq, int upper,
                  const uint64_t* part_offsets, uint32_t P, uint64_t* pos_out, uint32_t* part_out, void* stream) {
  const u32 w = key_width(key_type);
  if (!w) return fail(LBSORT_ERR_INVALID_ARG, "key_type must be one of LBSORT_U32..LBSORT_F64 (got %d)", key_type);
  if (upper != 0 && upper != 1) return fail(LBSORT_ERR_INVALID_ARG, "upper must be 0 or 1 (got %d)", upper);
  if (nq == 0) return LBSORT_OK;
  if (!queries || !pos_out) return fail(LBSORT_ERR_INVALID_ARG, "queries/pos_out must not be NULL");
  if (n > 0 && !sorted_keys) return fail(LBSORT_ERR_INVALID_ARG, "sorted_keys must not be NULL");
  if (part_out && (!part_offsets || P < 1 || P > LBSORT_MAX_P))
    return fail(LBSORT_ERR_INVALID_ARG, "part_out needs part_offsets and P in [1, %d]", LBSORT_MAX_P);
  if (nq / 256 >= (1ull << 31)) return fail(LBSORT_ERR_UNSUPPORTED, "too many queries in one call");
  u64 top, fm;
  key_masks(key_type, top, fm);
  hipStream_t st = (hipStream_t)stream;
  if (w == 8)
    launch_search<u64>((const u64*)sorted_keys, n, (const u64*)queries, nq, upper != 0, top, fm, part_offsets, P,
                       pos_out, part_out, st);
  else
    launch_search<u32>((const u32*)sorted_keys, n, (const u32*)queries, nq, upper != 0, top, fm, part_offsets, P,
                       pos_out, part_out, st);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return fail(LBSORT_ERR_HIP, "kernel launch failed: %s", hipGetErrorString(e));
  return LBSORT_OK;
}

uint64_t lbsort_search_index_bytes(int key_type, uint64_t n) {
  const u32 w = key_width(key_type);
  if (!w) return 0;
  return SearchIndexLayout(n, w).bytes;
}

int lbsort_search_build_index(int key_type, const void* sorted_keys, uint64_t n, void* index, void* stream) {
  const u32 w = key_width(key_type);
  if (!w) return fail(LBSORT_ERR_INVALID_ARG, "key_type must be one of LBSORT_U32..LBSORT_F64 (got %d)", key_type);
  const SearchIndexLayout lay(n, w);
  if (lay.bytes == 0) return LBSORT_OK;
  if (!sorted_keys || !index) return fail(LBSORT_ERR_INVALID_ARG, "sorted_keys/index must not be NULL");
  if ((uintptr_t)index % 128 != 0) return fail(LBSORT_ERR_INVALID_ARG, "index must be 128-byte aligned");
  hipStream_t st = (hipStream_t)stream;
  if (w == 8)
    launch_search_index_build<u64>((const u64*)sorted_keys, n, index, st);
  else
    launch_search_index_build<u32>((const u32*)sorted_keys, n, index, st);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return fail(LBSORT_ERR_HIP, "kernel launch failed: %s", hipGetErrorString(e));
  return LBSORT_OK;
}

int lbsort_search_indexed(int key_type, const void* sorted_keys, uint64_t n, const void* index, const void* queries,
                          uint64_t nq, int upper, const uint64_t* part_offsets, uint32_t P, uint64_t* pos_out,
                          uint32_t* part_out, void* stream) {
  const u32 w = key_width(key_type);
  if (!w) return fail(LBSORT_ERR_INVALID_ARG, "key_type must be one of LBSORT_U32..LBSORT_F64 (got %d)", key_type);
  if (upper != 0 && upper != 1) return fail(LBSORT_ERR_INVALID_ARG, "upper must be 0 or 1 (got %d)", upper);
  if (nq == 0) return LBSORT_OK;
  if (!queries || !pos_out) return fail(LBSORT_ERR_INVALID_ARG, "queries/pos_out must not be NULL");
  if (n > 0 && !sorted_keys) return fail(LBSORT_ERR_INVALID_ARG, "sorted_keys must not be NULL");
  if (SearchIndexLayout(n, w).bytes > 0 && !index)
    return fail(LBSORT_ERR_INVALID_ARG, "index must not be NULL for n > 16 (lbsort_search_build_index)");
  if (part_out && (!part_offsets || P < 1 || P > LBSORT_MAX_P))
    return fail(LBSORT_ERR_INVALID_ARG, "part_out needs part_offsets and P in [1, %d]", LBSORT_MAX_P);
  if (nq / 256 >= (1ull << 31)) return fail(LBSORT_ERR_UNSUPPORTED, "too many queries in one call");
  u64 top, fm;
  key_masks(key_type, top, fm);
  hipStream_t st = (hipStream_t)stream;
  if (w == 8)
    launch_search_indexed<u64>((const u64*)sorted_keys, n, index, (const u64*)queries, nq, upper != 0, top, fm,
                               part_offsets, P, pos_out, part_out, st);
  else
    launch_search_indexed<u32>((const u32*)sorted_keys, n, index, (const u32*)queries, nq, upper != 0, top, fm,
                               part_offsets, P, pos_out, part_out, st);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return fail(LBSORT_ERR_HIP, "kernel launch failed: %s", hipGetErrorString(e));
  return LBSORT_OK;
}

int lbsort_provenance(const uint32_t* src_index, uint64_t count, uint64_t n, uint32_t P, uint32_t* src_block,
                      uint32_t* src_offset, void* stream) {
  if (P < 1 || P > LBSORT_MAX_P) return fail(LBSORT_ERR_INVALID_ARG, "P must be in [1, %d] (got %u)", LBSORT_MAX_P, P);
  if (n > (1ull << 32)) return fail(LBSORT_ERR_UNSUPPORTED, "n must be <= 2^32 (32-bit positions)");
  if (count == 0) return LBSORT_OK;
  if (!src_index || (!src_block && !src_offset))
    return fail(LBSORT_ERR_INVALID_ARG, "src_index and one of src_block/src_offset must not be NULL");
  if (count / 256 >= (1ull << 31)) return fail(LBSORT_ERR_UNSUPPORTED, "too many entries in one call");
  launch_provenance(src_index, count, n, P, src_block, src_offset, (hipStream_t)stream);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return fail(LBSORT_ERR_HIP, "kernel launch failed: %s", hipGetErrorString(e));
  return LBSORT_OK;
}

int lbsort_check(void* ws, void* stream) {
  if (!ws) return fail(LBSORT_ERR_INVALID_ARG, "ws must not be NULL");
  hipError_t e = hipStreamSynchronize((hipStream_t)stream);
  if (e != hipSuccess) return fail(LBSORT_ERR_HIP, "stream synchronize failed: %s", hipGetErrorString(e));
  u32 err = 0;
  e = hipMemcpy(&err, (char*)ws + 0 + C_ERR * 4, 4, hipMemcpyDeviceToHost);
  if (e != hipSuccess) return fail(LBSORT_ERR_HIP, "reading the device error word failed: %s", hipGetErrorString(e));
  if (err) {
    const u32 zero = 0;
    hipMemcpy((char*)ws + C_ERR * 4, &zero, 4, hipMemcpyHostToDevice);
    return fail(LBSORT_ERR_DEVICE, "device error bits 0x%x (%s%s%s%s)", err, (err & E_SPIN) ? "look-back wait gave up " : "",
                (err & E_SEG) ? "malformed seg_offsets " : "", (err & E_SELECT) ? "merge selection did not converge " : "",
                (err & E_RANGE) ? "block of 2^32 keys or more" : "");
  }
  return LBSORT_OK;
}

const char* lbsort_status_string(int status) {
  switch (status) {
    case LBSORT_OK: return "ok";
    case LBSORT_ERR_INVALID_ARG: return "invalid argument";
    case LBSORT_ERR_WORKSPACE_TOO_SMALL: return "workspace too small";
    case LBSORT_ERR_UNSUPPORTED: return "unsupported";
    case LBSORT_ERR_HIP: return "HIP runtime error";
    case LBSORT_ERR_OOM: return "out of device memory";
    case LBSORT_ERR_DEVICE: return "error detected on the device";
    default: return "unknown status";
  }
}

const char* lbsort_last_error(void) { return g_last_error.c_str(); }

}  // extern "C"
