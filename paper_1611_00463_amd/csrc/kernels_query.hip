// Queries over a sorted result (Section III and Section IV.C): binary search
// of many keys at once, the processor and index each sorted entry came from,
// and the in-place map of sorted keys back to a signed or float type.
#include "lbsort_internal.hpp"

namespace lbs {

// In place: keys of the order-preserving unsigned image back to their type.
template <typename K>
__global__ __launch_bounds__(256) void k_key_out(K* __restrict__ a, u64 n, u64 top, u64 fm) {
  const u64 stride = (u64)gridDim.x * 256;
  for (u64 i = (u64)blockIdx.x * 256 + threadIdx.x; i < n; i += stride) a[i] = key_out<K>(a[i], top, fm);
}

// One query per thread.  pos = number of keys below the query (or not above
// it, UPPER), both compared through the order-preserving map (top, fm), so
// the same loop serves every key type.  part = the partition k with
// G_k <= pos < G_{k+1}, P when pos = n.
template <typename K, bool UPPER>
__global__ __launch_bounds__(256) void k_search(const K* __restrict__ a, u64 n, const K* __restrict__ q, u64 nq,
                                                u64 top, u64 fm, const u64* __restrict__ G, u32 P,
                                                u64* __restrict__ pos_out, u32* __restrict__ part_out) {
  const u64 j = (u64)blockIdx.x * 256 + threadIdx.x;
  if (j >= nq) return;
  const K x = key_in<K>(q[j], top, fm);
  u64 lo = 0, len = n;
  while (len > 0) {
    const u64 half = len >> 1;
    const K v = key_in<K>(a[lo + half], top, fm);
    if (UPPER ? v <= x : v < x) {
      lo += half + 1;
      len -= half + 1;
    } else {
      len = half;
    }
  }
  pos_out[j] = lo;
  if (part_out) {
    u32 k = P;
    if (lo < n) {
      // largest k in [0, P) with G_k <= lo (G_0 = 0 <= lo < n = G_P)
      u32 a0 = 0, b0 = P;
      while (b0 - a0 > 1) {
        const u32 mid = (a0 + b0) >> 1;
        if (G[mid] <= lo) a0 = mid; else b0 = mid;
      }
      k = a0;
    }
    part_out[j] = k;
  }
}

// Search index (layout: SearchIndexLayout): one thread per index key, all
// levels at once, each read straight from the sorted array (the key at
// position i * 16^l).
template <typename K>
__global__ __launch_bounds__(256) void k_search_index_build(const K* __restrict__ a, SearchIndexLayout lay,
                                                            char* __restrict__ index, u64 total) {
  const u64 stride = (u64)gridDim.x * 256;
  for (u64 e = (u64)blockIdx.x * 256 + threadIdx.x; e < total; e += stride) {
    int l = 1;
    u64 i = e, span = SI_FAN;
    while (i >= lay.n[l]) {
      i -= lay.n[l];
      ++l;
      span *= SI_FAN;
    }
    ((K*)(index + lay.off[l]))[i] = a[i * span];
  }
}

// Count of the keys of group [base, base + cnt) of a level below the query
// (or not above it, UPPER): a binary search inside one 128-byte group.
template <typename K, bool UPPER>
__device__ inline u64 group_count(const K* lvl, u64 base, u32 cnt, K x, u64 top, u64 fm) {
  u32 lo = 0, len = cnt;
  while (len > 0) {
    const u32 half = len >> 1;
    const K v = key_in<K>(lvl[base + lo + half], top, fm);
    if (UPPER ? v <= x : v < x) {
      lo += half + 1;
      len -= half + 1;
    } else {
      len = half;
    }
  }
  return base + lo;
}

// One query per thread over the index: the count at the top level (at most
// 16 keys), then one group of 16 keys per level down to the sorted array.
// The count of level l is ceil(c / 16^l) for the array's count c, so the
// count of level l - 1 lies in group c_l - 1 of that level (and is 0 when
// c_l is).  About one cache line per level instead of one per halving.
template <typename K, bool UPPER>
__global__ __launch_bounds__(256) void k_search_indexed(const K* __restrict__ a, SearchIndexLayout lay,
                                                        const char* __restrict__ index, const K* __restrict__ q, u64 nq,
                                                        u64 top, u64 fm, const u64* __restrict__ G, u32 P,
                                                        u64* __restrict__ pos_out, u32* __restrict__ part_out) {
  const u64 j = (u64)blockIdx.x * 256 + threadIdx.x;
  if (j >= nq) return;
  const u64 n = lay.n[0];
  const K x = key_in<K>(q[j], top, fm);
  auto level = [&](int l) -> const K* { return l == 0 ? a : (const K*)(index + lay.off[l]); };
  u64 c = group_count<K, UPPER>(level(lay.top), 0, (u32)lay.n[lay.top], x, top, fm);
  for (int l = lay.top; l >= 1 && c > 0; --l) {
    const u64 base = (c - 1) * SI_FAN;
    const u64 left = lay.n[l - 1] - base;
    c = group_count<K, UPPER>(level(l - 1), base, (u32)(left < SI_FAN ? left : SI_FAN), x, top, fm);
  }
  pos_out[j] = c;
  if (part_out) {
    u32 k = P;
    if (c < n) {
      // largest k in [0, P) with G_k <= c (G_0 = 0 <= c < n = G_P)
      u32 a0 = 0, b0 = P;
      while (b0 - a0 > 1) {
        const u32 mid = (a0 + b0) >> 1;
        if (G[mid] <= c) a0 = mid; else b0 = mid;
      }
      k = a0;
    }
    part_out[j] = k;
  }
}

// Input position g of n keys split into P equal blocks (block i holds
// [floor(i n / P), floor((i+1) n / P))): its block is the largest i with
// floor(i n / P) <= g, i.e. i n < (g + 1) P, so i = ceil((g + 1) P / n) - 1.
// Positions >= n give block 0xFFFFFFFF and offset 0xFFFFFFFF.
__global__ __launch_bounds__(256) void k_provenance(const u32* __restrict__ idx, u64 count, u64 n, u32 P,
                                                   u32* __restrict__ blk_out, u32* __restrict__ off_out) {
  const u64 j = (u64)blockIdx.x * 256 + threadIdx.x;
  if (j >= count) return;
  const u64 g = idx[j];
  u32 b = 0xFFFFFFFFu, o = 0xFFFFFFFFu;
  if (g < n) {
    b = (u32)(((g + 1) * P - 1) / n);
    o = (u32)(g - ((u64)b * n) / P);
  }
  if (blk_out) blk_out[j] = b;
  if (off_out) off_out[j] = o;
}

template <typename K>
void launch_key_out(K* a, u64 n, u64 top, u64 fm, hipStream_t s) {
  if (n == 0) return;
  const u64 want = (n + 255) / 256;
  const u32 grid = (u32)(want < 65536 ? want : 65536);
  { const int pe_ = prof_begin(s); hipLaunchKernelGGL(k_key_out<K>, dim3(grid), dim3(256), 0, s, a, n, top, fm); prof_end(pe_, "key_out", s); }
}

template <typename K>
void launch_search(const K* a, u64 n, const K* q, u64 nq, bool upper, u64 top, u64 fm, const u64* G, u32 P,
                   u64* pos, u32* part, hipStream_t s) {
  if (nq == 0) return;
  const dim3 grid((u32)((nq + 255) / 256));
  const int pe_ = prof_begin(s);
  if (upper)
    hipLaunchKernelGGL((k_search<K, true>), grid, dim3(256), 0, s, a, n, q, nq, top, fm, G, P, pos, part);
  else
    hipLaunchKernelGGL((k_search<K, false>), grid, dim3(256), 0, s, a, n, q, nq, top, fm, G, P, pos, part);
  prof_end(pe_, "search", s);
}

template <typename K>
void launch_search_index_build(const K* a, u64 n, void* index, hipStream_t s) {
  const SearchIndexLayout lay(n, sizeof(K));
  u64 total = 0;
  for (int l = 1; l <= lay.top; ++l) total += lay.n[l];
  if (total == 0) return;
  const u64 want = (total + 255) / 256;
  const u32 grid = (u32)(want < 65536 ? want : 65536);
  const int pe_ = prof_begin(s);
  hipLaunchKernelGGL(k_search_index_build<K>, dim3(grid), dim3(256), 0, s, a, lay, (char*)index, total);
  prof_end(pe_, "search_index", s);
}

template <typename K>
void launch_search_indexed(const K* a, u64 n, const void* index, const K* q, u64 nq, bool upper, u64 top, u64 fm,
                           const u64* G, u32 P, u64* pos, u32* part, hipStream_t s) {
  if (nq == 0) return;
  const SearchIndexLayout lay(n, sizeof(K));
  const dim3 grid((u32)((nq + 255) / 256));
  const int pe_ = prof_begin(s);
  if (upper)
    hipLaunchKernelGGL((k_search_indexed<K, true>), grid, dim3(256), 0, s, a, lay, (const char*)index, q, nq, top, fm,
                       G, P, pos, part);
  else
    hipLaunchKernelGGL((k_search_indexed<K, false>), grid, dim3(256), 0, s, a, lay, (const char*)index, q, nq, top,
                       fm, G, P, pos, part);
  prof_end(pe_, "search_indexed", s);
}

void launch_provenance(const u32* idx, u64 count, u64 n, u32 P, u32* blk, u32* off, hipStream_t s) {
  if (count == 0) return;
  const int pe_ = prof_begin(s);
  hipLaunchKernelGGL(k_provenance, dim3((u32)((count + 255) / 256)), dim3(256), 0, s, idx, count, n, P, blk, off);
  prof_end(pe_, "provenance", s);
}

template void launch_key_out<u32>(u32*, u64, u64, u64, hipStream_t);
template void launch_key_out<u64>(u64*, u64, u64, u64, hipStream_t);
template void launch_search<u32>(const u32*, u64, const u32*, u64, bool, u64, u64, const u64*, u32, u64*, u32*, hipStream_t);
template void launch_search<u64>(const u64*, u64, const u64*, u64, bool, u64, u64, const u64*, u32, u64*, u32*, hipStream_t);

template void launch_search_index_build<u32>(const u32*, u64, void*, hipStream_t);
template void launch_search_index_build<u64>(const u64*, u64, void*, hipStream_t);
template void launch_search_indexed<u32>(const u32*, u64, const void*, const u32*, u64, bool, u64, u64, const u64*, u32,
                                         u64*, u32*, hipStream_t);
template void launch_search_indexed<u64>(const u64*, u64, const void*, const u64*, u64, bool, u64, u64, const u64*, u32,
                                         u64*, u32*, hipStream_t);

}  // namespace lbs
