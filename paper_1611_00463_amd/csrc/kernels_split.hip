// Steps 2-5 of Section IV on the GPU: regular samples of the sorted blocks,
// splitters chosen from the pooled samples, binary search of every splitter
// in every block, the investigator that divides runs of keys equal to a
// splitter, and the range table (send counts and receive offsets) that the
// exchange and the merge use.  All of it is a few kilobytes of metadata;
// nothing here touches the bulk of the data except the searches.
#include "lbsort_internal.hpp"
#include "select.hpp"

namespace lbs {

// Step 2: s_i = min(s, n_i) regular samples of sorted block i at the chunk
// starts floor(j n_i / s_i) (the regular sampling of PSRS).
template <typename K>
__global__ __launch_bounds__(256) void k_samples(Plan p, const K* __restrict__ sorted, u64 max_samples) {
  __shared__ u32 s_rng[2];
  const u64 x0 = (u64)blockIdx.x * 256, x = x0 + threadIdx.x;
  const u64 total = min(max_samples, (u64)p.samp_start[p.NB]);
  if (x0 >= total) return;  // the whole workgroup
  const u32 blk = wg_find_seg(p.samp_start, p.NB, x, x0, min(x0 + 255, total - 1), s_rng);
  if (x >= total) return;
  const u64 j = x - p.samp_start[blk];
  const u64 si = p.samp_start[blk + 1] - p.samp_start[blk];
  const u64 bs = p.blk_start[blk];
  const u64 n = p.blk_start[blk + 1] - bs;
  // j < si <= n < 2^32 (the plan bounds block sizes), so j n fits 64 bits
  const u64 pos = j * n / si;
  ((K*)p.samples)[x] = sorted[bs + pos];
}

// Step 3, part 1: the rank of every sample in its instance's pool, where
// equal keys are ordered by (block, position).  A group of G lanes counts, in
// every other block's sample list, the samples that precede this one; the
// sample is then stored at its rank, which sorts the pool.
template <typename K, int G>
__global__ __launch_bounds__(256) void k_sample_rank(Plan p, u64 max_samples) {
  const u64 gid = ((u64)blockIdx.x * blockDim.x + threadIdx.x) / G;
  const u32 sub = threadIdx.x % G;
  const bool live = gid < max_samples && gid < p.samp_start[p.NB];
  u64 cnt = 0;
  u64 dst = 0;
  K key = 0;
  if (live) {
    const u32 blk = find_seg(p.samp_start, p.NB, gid);
    const u32 b = blk / p.P, i = blk % p.P;
    const K* smp = (const K*)p.samples;
    key = smp[gid];
    for (u32 o = sub; o < p.P; o += G) {
      if (o == i) continue;
      const u64 a = p.samp_start[b * p.P + o], e = p.samp_start[b * p.P + o + 1];
      cnt += (o < i) ? bsearch_count<K, true>(smp, a, e, key) - a : bsearch_count<K, false>(smp, a, e, key) - a;
    }
    dst = p.samp_start[b * p.P] + (gid - p.samp_start[blk]);
  }
#pragma unroll
  for (int o = G / 2; o > 0; o >>= 1) cnt += __shfl_xor(cnt, o, G);
  if (live && sub == 0) ((K*)p.pool)[dst + cnt] = key;
}

// Step 3, part 2: splitter k = pool[min(S-1, floor(k S / P) + floor(P/2) - 1)],
// the middle of the k-th group of P pooled samples (PSRS's pivot rank).
template <typename K>
__global__ __launch_bounds__(256) void k_splitters(Plan p) {
  const u32 x = blockIdx.x * blockDim.x + threadIdx.x;
  const u32 per = p.P - 1;
  if (x >= p.B * per) return;
  const u32 b = x / per, k = x % per + 1;
  const u64 a = p.samp_start[b * p.P], S = p.samp_start[(b + 1) * p.P] - a;
  K v = key_in<K>((K)0, p.ky_top, p.ky_fm);  // no samples: the key type's zero
  if (S > 0) {
    const u64 r = ((u64)k * S) / p.P + p.P / 2 - 1;
    v = ((const K*)p.pool)[a + (r < S - 1 ? r : S - 1)];
  }
  ((K*)p.splitters)[x] = v;
}

// Step 3 for P <= 16: splitter k is the element of rank t_k of the union of
// the P sorted sample lists of its instance, found by the wave-wide
// multi-sequence selection (one wave per splitter) without ranking every
// sample: the element of rank t is the smallest first element beyond the split
// of the first t elements.
template <typename K, int F>
__global__ __launch_bounds__(256) void k_select_splitters(Plan p) {
  const u32 wv = (blockIdx.x * blockDim.x + threadIdx.x) >> 6;
  const u32 lane = threadIdx.x & 63;
  const u32 per = p.P - 1;
  if (wv >= p.B * per) return;
  const u32 b = wv / per, k = wv % per + 1;
  const u32 r = lane % F;
  const u64 a0 = p.samp_start[b * p.P];
  const u64 S = p.samp_start[(b + 1) * p.P] - a0;
  K v = key_in<K>((K)0, p.ky_top, p.ky_fm);  // no samples: the key type's zero
  if (S > 0) {
    const u64 t0 = ((u64)k * S) / p.P + p.P / 2 - 1;
    const u64 t = t0 < S - 1 ? t0 : S - 1;
    u64 roff = 0, rlen = 0;
    if (r < p.P) {
      roff = p.samp_start[b * p.P + r];
      rlen = p.samp_start[b * p.P + r + 1] - roff;
    }
    const u64 lo = t + rlen > S ? t + rlen - S : 0;
    const u64 hi = t < rlen ? t : rlen;
    const K* smp = (const K*)p.samples;
    const u64 cut = wave_select<K, F, F == 16 ? 8 : (F == 8 ? 4 : (F == 4 ? 2 : 1))>(smp, roff, lo, hi, t, p.counters);
    // smallest key among the run fronts just past the split
    bool has = cut < rlen;
    K front = has ? smp[roff + cut] : (K)0;
#pragma unroll
    for (int o = 1; o < F; o <<= 1) {
      const K of = __shfl_xor(front, o);
      const bool oh = __shfl_xor((int)has, o) != 0;
      if (oh && (!has || of < front)) front = of;
      has = has || oh;
    }
    v = front;
  }
  if (lane == 0) ((K*)p.splitters)[(u64)b * per + k - 1] = v;
}

// Step 4: lo = #keys < v_k and hi = #keys <= v_k in every sorted block.  The
// block's own samples (sorted, at known positions) narrow the window before
// the search in the block itself.
template <typename K>
__global__ __launch_bounds__(256) void k_search(Plan p, const K* __restrict__ sorted) {
  const u32 x = blockIdx.x * blockDim.x + threadIdx.x;
  const u32 per = p.P - 1;
  if (x >= p.B * p.P * per * 2) return;
  const bool upper = x & 1;
  const u32 y = x >> 1;
  const u32 blk = y / per, k = y % per;
  const u32 b = blk / p.P;
  const K v = ((const K*)p.splitters)[b * per + k];
  const u64 bs = p.blk_start[blk], n = p.blk_start[blk + 1] - bs;
  // window from the samples: sample j sits at floor(j n / si)
  const u64 sa = p.samp_start[blk], si = p.samp_start[blk + 1] - sa;
  const K* smp = (const K*)p.samples;
  u64 wlo = 0, whi = n;
  if (si > 0) {
    const u64 j = upper ? bsearch_count<K, true>(smp, sa, sa + si, v) - sa : bsearch_count<K, false>(smp, sa, sa + si, v) - sa;
    // j <= si <= n < 2^32: the products fit 64 bits
    if (j > 0) wlo = (j - 1) * n / si + 1;
    if (j < si) whi = j * n / si;
  }
  const u64 r = upper ? bsearch_count<K, true>(sorted + bs, wlo, whi, v) : bsearch_count<K, false>(sorted + bs, wlo, whi, v);
  (upper ? p.hi : p.lo)[(u64)blk * per + k] = r;
}

// Step 4, the investigator, and the range table of step 5.  One workgroup per
// instance, one thread per splitter k.
//  COUNT: L_k = sum_i lo, H_k = sum_i hi, G_k = clamp(floor(kN/P), L_k, H_k);
//         the G_k - L_k keys equal to v_k that partition k-1 still needs are
//         taken from the blocks in block order.
//  NONE:  cut = lo.
//  PAPER: for d equal splitters, each block's equal range is cut into d+1
//         equal pieces.
template <typename K>
__global__ __launch_bounds__(1024) void k_investigate(Plan p, u64* __restrict__ out_offsets,
                                                      u64* __restrict__ out_counts, u64* __restrict__ out_send,
                                                      u64* __restrict__ out_cuts, K* __restrict__ out_split) {
  const u32 b = blockIdx.x;
  const u32 P = p.P, per = P - 1;
  const u64 N = p.seg[b + 1] - p.seg[b];
  // the loops over the P blocks take 8 blocks at a time, loads before
  // stores, so that 8 loads are in flight rather than one
  u64* cuts = p.cuts + (u64)b * P * (P + 1);
  const u64* lo = p.lo + (u64)b * P * per;
  const u64* hi = p.hi + (u64)b * P * per;
  const K* v = (const K*)p.splitters + (u64)b * per;
  const u32 blk0 = b * P;
  for (u32 k = threadIdx.x; k <= P; k += blockDim.x) {
    if (k == 0 || k == P || p.inv == 1) {
      // column 0 (zero), column P (the block sizes), NONE (the lower bounds)
      for (u32 i0 = 0; i0 < P; i0 += 8) {
        u64 c[8];
#pragma unroll
        for (u32 u = 0; u < 8; ++u) {
          const u32 i = i0 + u < P ? i0 + u : P - 1;
          c[u] = k == 0 ? 0 : (k == P ? p.blk_start[blk0 + i + 1] - p.blk_start[blk0 + i] : lo[(u64)i * per + k - 1]);
        }
#pragma unroll
        for (u32 u = 0; u < 8; ++u)
          if (i0 + u < P) cuts[(u64)(i0 + u) * (P + 1) + k] = c[u];
      }
    } else if (p.inv == 2) {
      for (u32 i = 0; i < P; ++i) {
        // run of equal splitters containing k: [k0, k0 + d)
        u32 k0 = k;
        while (k0 > 1 && v[k0 - 2] == v[k - 1]) --k0;
        u32 d = 1;
        while (k0 + d < P && v[k0 + d - 1] == v[k0 - 1]) ++d;
        const u64 base = lo[(u64)i * per + k0 - 1];
        const u64 m = hi[(u64)i * per + k0 - 1] - base;
        cuts[(u64)i * (P + 1) + k] = d == 1 ? base : base + ((u64)(k - k0 + 1) * m) / (d + 1);
      }
    }
    if (k > 0 && k < P && p.inv == 0) {
      u64 L = 0, H = 0;
#pragma unroll 8
      for (u32 i = 0; i < P; ++i) {
        L += lo[(u64)i * per + k - 1];
        H += hi[(u64)i * per + k - 1];
      }
      // k <= P <= 1024: below 2^53 keys k N fits 64 bits
      const u64 T = N < (1ull << 53) ? (u64)k * N / P : (u64)(((unsigned __int128)k * N) / P);
      const u64 Gk = T < L ? L : (T > H ? H : T);
      u64 extra = Gk - L;
      for (u32 i0 = 0; i0 < P; i0 += 8) {
        // a chunk's loads first, then its stores
        u64 l[8], h[8];
#pragma unroll
        for (u32 u = 0; u < 8; ++u) {
          const u32 i = i0 + u < P ? i0 + u : P - 1;
          l[u] = lo[(u64)i * per + k - 1];
          h[u] = hi[(u64)i * per + k - 1];
        }
#pragma unroll
        for (u32 u = 0; u < 8; ++u) {
          if (i0 + u >= P) break;
          const u64 m = h[u] - l[u];
          const u64 take = m < extra ? m : extra;
          extra -= take;
          cuts[(u64)(i0 + u) * (P + 1) + k] = l[u] + take;
        }
      }
    }
  }
  __syncthreads();
  // Range table: C[i][k], G_k, receive offsets D[i][k] = G_k + sum_{i'<i} C[i'][k].
  u64* Gb = p.G + (u64)b * (P + 1);
  u64* Db = p.Dm + (u64)b * (P + 1) * P;
  for (u32 k = threadIdx.x; k <= P; k += blockDim.x) {
    u64 g = 0;
#pragma unroll 8
    for (u32 i = 0; i < P; ++i) g += cuts[(u64)i * (P + 1) + k];
    Gb[k] = g;
    out_offsets[(u64)b * (P + 1) + k] = g;
  }
  __syncthreads();
  for (u32 k = threadIdx.x; k < P; k += blockDim.x) {
    u64 acc = Gb[k];
    for (u32 i0 = 0; i0 < P; i0 += 8) {
      // a chunk's loads first, then its stores
      u64 c[8];
#pragma unroll
      for (u32 u = 0; u < 8; ++u) {
        const u32 i = i0 + u < P ? i0 + u : P - 1;
        c[u] = cuts[(u64)i * (P + 1) + k + 1] - cuts[(u64)i * (P + 1) + k];
      }
#pragma unroll
      for (u32 u = 0; u < 8; ++u) {
        if (i0 + u >= P) break;
        const u32 i = i0 + u;
        Db[(u64)i * P + k] = acc;
        acc += c[u];
        if (out_send) out_send[(u64)b * P * P + (u64)i * P + k] = c[u];
      }
    }
    Db[(u64)P * P + k] = Gb[k + 1];
    if (out_counts) out_counts[(u64)b * P + k] = Gb[k + 1] - Gb[k];
  }
  if (out_cuts)
    for (u32 x = threadIdx.x; x < P * (P + 1); x += blockDim.x) out_cuts[(u64)b * P * (P + 1) + x] = cuts[x];
  if (out_split)
    for (u32 x = threadIdx.x; x < per; x += blockDim.x) out_split[(u64)b * per + x] = key_out<K>(v[x], p.ky_top, p.ky_fm);
}

// ----------------------------------------------------------------- launchers
template <typename K>
void launch_split(const Plan& p, const K* sorted, u64 max_samples, const void* out_offsets_v,
                  void* out_counts, void* out_send, void* out_cuts, void* out_split, hipStream_t s) {
  if (p.P > 1 && max_samples > 0) {
    { const int pe_ = prof_begin(s); hipLaunchKernelGGL(k_samples<K>, dim3((u32)((max_samples + 255) / 256)), dim3(256), 0, s, p, sorted,
                       max_samples); prof_end(pe_, "samples", s); }
  }
  if (p.P > 1 && p.P <= 16) {
    const u32 waves = p.B * (p.P - 1);
    const dim3 grid((waves + 3) / 4);
    const int pe_ = prof_begin(s);
    if (p.P <= 2) hipLaunchKernelGGL((k_select_splitters<K, 2>), grid, dim3(256), 0, s, p);
    else if (p.P <= 4) hipLaunchKernelGGL((k_select_splitters<K, 4>), grid, dim3(256), 0, s, p);
    else if (p.P <= 8) hipLaunchKernelGGL((k_select_splitters<K, 8>), grid, dim3(256), 0, s, p);
    else hipLaunchKernelGGL((k_select_splitters<K, 16>), grid, dim3(256), 0, s, p);
    prof_end(pe_, "select_splitters", s);
  } else if (p.P > 16 && max_samples > 0) {
    const u32 G = p.P >= 64 ? 64 : (p.P >= 32 ? 32 : (p.P >= 16 ? 16 : (p.P >= 8 ? 8 : (p.P >= 4 ? 4 : 2))));
    const u64 threads = max_samples * G;
    const dim3 grid((u32)((threads + 255) / 256));
    const int pe_rank = prof_begin(s);
    switch (G) {
      case 64: hipLaunchKernelGGL((k_sample_rank<K, 64>), grid, dim3(256), 0, s, p, max_samples); break;
      case 32: hipLaunchKernelGGL((k_sample_rank<K, 32>), grid, dim3(256), 0, s, p, max_samples); break;
      case 16: hipLaunchKernelGGL((k_sample_rank<K, 16>), grid, dim3(256), 0, s, p, max_samples); break;
      case 8: hipLaunchKernelGGL((k_sample_rank<K, 8>), grid, dim3(256), 0, s, p, max_samples); break;
      case 4: hipLaunchKernelGGL((k_sample_rank<K, 4>), grid, dim3(256), 0, s, p, max_samples); break;
      default: hipLaunchKernelGGL((k_sample_rank<K, 2>), grid, dim3(256), 0, s, p, max_samples); break;
    }
    prof_end(pe_rank, "sample_rank", s);
  }
  if (p.P > 1) {
    const u32 ns = p.B * (p.P - 1);
    if (p.P > 16) { const int pe_ = prof_begin(s); hipLaunchKernelGGL(k_splitters<K>, dim3((ns + 255) / 256), dim3(256), 0, s, p); prof_end(pe_, "splitters", s); }
    const u64 nq = (u64)p.B * p.P * (p.P - 1) * 2;
    { const int pe_ = prof_begin(s); hipLaunchKernelGGL(k_search<K>, dim3((u32)((nq + 255) / 256)), dim3(256), 0, s, p, sorted); prof_end(pe_, "search", s); }
  }
  const u32 nt = p.P + 1 < 1024 ? ((p.P + 1 + 63) / 64) * 64 : 1024;
  { const int pe_ = prof_begin(s); hipLaunchKernelGGL(k_investigate<K>, dim3(p.B), dim3(nt), 0, s, p, (u64*)out_offsets_v, (u64*)out_counts,
                     (u64*)out_send, (u64*)out_cuts, (K*)out_split); prof_end(pe_, "investigate", s); }
}

template void launch_split<u32>(const Plan&, const u32*, u64, const void*, void*, void*, void*, void*, hipStream_t);
template void launch_split<u64>(const Plan&, const u64*, u64, const void*, void*, void*, void*, void*, hipStream_t);

}  // namespace lbs
