// Autotuner: picks the radix tile of the local sort, the handler's schedule
// (F-way passes or one sampled pass), its fan-in F and its merge tile for one
// shape by timing the candidates on the device
// (on the caller's own data, or on synthetic uniform instances), checks that
// every candidate produced the same bytes as the first, and keeps the winner
// in an in-process table keyed by the device architecture, which can be
// saved to / loaded from a small JSON file.
#include <hip/hip_runtime.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/lbsort.h"
#include "tuning.hpp"

namespace lbs {

struct Entry {
  std::string arch;  // e.g. "gfx950"
  uint32_t key_bytes, values, size_log2, batched, P, fanin, merge_tile, radix_tile, handler, presorted;
  double ms;
};

static std::mutex g_mu;
static std::vector<Entry> g_table;
static bool g_env_loaded = false;

static uint32_t size_class(uint64_t n) {
  uint32_t c = 0;
  while (c < 63 && (1ull << (c + 1)) <= n) ++c;
  return c;
}

static uint32_t key_bytes_of(int key_type) {
  switch (key_type) {
    case LBSORT_U32: case LBSORT_I32: case LBSORT_F32: return 4;
    case LBSORT_U64: case LBSORT_I64: case LBSORT_F64: return 8;
    default: return 0;
  }
}

// Architecture name of the current device ("gfx950"), cached per device; ""
// when there is no device.
static std::string current_arch() {
  constexpr int MAXD = 64;
  static std::mutex mu;
  static std::string names[MAXD];
  static bool have[MAXD];
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= MAXD) {
    (void)hipGetLastError();
    return "";
  }
  std::lock_guard<std::mutex> lk(mu);
  if (!have[dev]) {
    hipDeviceProp_t pr;
    if (hipGetDeviceProperties(&pr, dev) == hipSuccess) {
      const std::string a = pr.gcnArchName;
      names[dev] = a.substr(0, a.find(':'));
    }
    have[dev] = true;
  }
  return names[dev];
}

static int parse_file(const char* path, std::vector<Entry>& out) {
  FILE* f = fopen(path, "r");
  if (!f) return -1;
  std::string s;
  char buf[4096];
  size_t r;
  while ((r = fread(buf, 1, sizeof buf, f)) > 0) s.append(buf, r);
  fclose(f);
  // One object per entry: {"arch": "..", "key_bytes": .., "values": .., "size_log2": .., "batched": ..,
  // "P": .., "fanin": .., "merge_tile": .., "radix_tile": .., "handler": .., "presorted": .., "ms": ..}
  size_t pos = 0;
  while ((pos = s.find('{', pos + 1)) != std::string::npos) {
    size_t end = s.find('}', pos);
    if (end == std::string::npos) break;
    std::string obj = s.substr(pos, end - pos);
    auto num = [&](const char* name, double& v) {
      std::string pat = std::string("\"") + name + "\":";
      size_t p = obj.find(pat);
      if (p == std::string::npos) return false;
      v = strtod(obj.c_str() + p + pat.size(), nullptr);
      return true;
    };
    auto str = [&](const char* name, std::string& v) {
      std::string pat = std::string("\"") + name + "\": \"";
      size_t p = obj.find(pat);
      if (p == std::string::npos) return false;
      size_t q = obj.find('"', p + pat.size());
      if (q == std::string::npos) return false;
      v = obj.substr(p + pat.size(), q - p - pat.size());
      return true;
    };
    std::string arch;
    double kb, vt, sl, b, P, F, T, R, H, S, ms = 0;
    if (str("arch", arch) && num("key_bytes", kb) && num("values", vt) && num("size_log2", sl) &&
        num("batched", b) && num("P", P) && num("fanin", F) && num("merge_tile", T) && num("radix_tile", R) &&
        num("handler", H) && num("presorted", S)) {
      num("ms", ms);
      out.push_back(Entry{arch, (uint32_t)kb, (uint32_t)vt, (uint32_t)sl, (uint32_t)b, (uint32_t)P, (uint32_t)F,
                          (uint32_t)T, (uint32_t)R, (uint32_t)H, (uint32_t)S, ms});
    }
    pos = end;
  }
  return 0;
}

static int write_file(const char* path) {
  FILE* f = fopen(path, "w");
  if (!f) return -1;
  fprintf(f, "{\"entries\": [\n");
  for (size_t i = 0; i < g_table.size(); ++i) {
    const Entry& e = g_table[i];
    fprintf(f,
            "  {\"arch\": \"%s\", \"key_bytes\": %u, \"values\": %u, \"size_log2\": %u, \"batched\": %u, \"P\": %u, "
            "\"fanin\": %u, \"merge_tile\": %u, \"radix_tile\": %u, \"handler\": %u, \"presorted\": %u, "
            "\"ms\": %.4f}%s\n",
            e.arch.c_str(), e.key_bytes, e.values, e.size_log2, e.batched, e.P, e.fanin, e.merge_tile, e.radix_tile,
            e.handler, e.presorted, e.ms, i + 1 < g_table.size() ? "," : "");
  }
  fprintf(f, "]}\n");
  fclose(f);
  return 0;
}

static void upsert(const Entry& e) {
  for (auto& x : g_table)
    if (x.arch == e.arch && x.key_bytes == e.key_bytes && x.values == e.values && x.size_log2 == e.size_log2 &&
        x.batched == e.batched && x.P == e.P) {
      x = e;
      return;
    }
  g_table.push_back(e);
}

Tuned tuning_lookup(uint32_t key_bytes, bool values, uint64_t n, uint32_t B, uint32_t P) {
  const std::string arch = current_arch();
  std::lock_guard<std::mutex> lk(g_mu);
  if (!g_env_loaded) {
    g_env_loaded = true;
    const char* env = getenv("LBSORT_TUNE_CACHE");
    if (env && *env) {
      std::vector<Entry> v;
      if (parse_file(env, v) == 0)
        for (auto& e : v) upsert(e);
    }
  }
  Tuned t = {0, 0, 0, 0, 0};
  if (arch.empty()) return t;
  const uint32_t sc = size_class(n);
  const uint32_t batched = B > 1 ? 1 : 0;
  const Entry* best = nullptr;
  for (auto& e : g_table) {
    if (e.arch != arch || e.key_bytes != key_bytes || e.values != (values ? 1u : 0u) || e.batched != batched ||
        e.P != P)
      continue;
    if (!best || (uint32_t)abs((int)e.size_log2 - (int)sc) < (uint32_t)abs((int)best->size_log2 - (int)sc)) best = &e;
  }
  if (best && (uint32_t)abs((int)best->size_log2 - (int)sc) <= 2) {
    t.fanin = best->fanin;
    t.merge_tile = best->merge_tile;
    t.radix_tile = best->radix_tile;
    t.handler = best->handler;
    t.presorted = best->presorted;
  }
  return t;
}

// Synthetic instances: SplitMix64 (Steele, Lea and Flood 2014) of the index.
__global__ void k_gen(void* keys, uint32_t* vals, uint64_t n, int key64, uint64_t seed) {
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (uint64_t)gridDim.x * blockDim.x) {
    uint64_t z = seed + (i + 1) * 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    z ^= z >> 31;
    if (key64) ((uint64_t*)keys)[i] = z;
    else ((uint32_t*)keys)[i] = (uint32_t)(z >> 32);
    if (vals) vals[i] = (uint32_t)i;
  }
}

// Number of 32-bit words that differ between a and b, added to *count.
__global__ void k_diff(const uint32_t* a, const uint32_t* b, uint64_t words, unsigned long long* count) {
  unsigned long long c = 0;
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < words; i += (uint64_t)gridDim.x * blockDim.x)
    c += a[i] != b[i] ? 1 : 0;
  if (c) atomicAdd(count, c);
}

}  // namespace lbs

using namespace lbs;

extern "C" int lbsort_load_tuning(const char* cache_path) {
  if (!cache_path) return LBSORT_ERR_INVALID_ARG;
  std::vector<Entry> v;
  if (parse_file(cache_path, v) != 0) return LBSORT_ERR_INVALID_ARG;
  std::lock_guard<std::mutex> lk(g_mu);
  g_env_loaded = true;
  for (auto& e : v) upsert(e);
  return LBSORT_OK;
}

extern "C" int lbsort_autotune(int key_type, int val_type, const void* keys_in, const void* vals_in,
                               const uint64_t* seg_offsets, uint32_t B, uint64_t total_n, uint32_t P,
                               const char* cache_path, lbsort_params* chosen) {
  const uint64_t kb = key_bytes_of(key_type);
  if (!kb || (val_type != LBSORT_NOVAL && val_type != LBSORT_VAL_U32 && val_type != LBSORT_VAL_INDEX) ||
      total_n == 0 || B == 0 || P < 1 || P > LBSORT_MAX_P)
    return LBSORT_ERR_INVALID_ARG;
  if (keys_in && B > 1 && !seg_offsets) return LBSORT_ERR_INVALID_ARG;
  if (keys_in && val_type == LBSORT_VAL_U32 && !vals_in) return LBSORT_ERR_INVALID_ARG;
  const std::string arch = current_arch();
  if (arch.empty()) return LBSORT_ERR_HIP;
  const bool hasv = val_type != LBSORT_NOVAL;
  // candidates: radix tile x handler schedule (each exact fan-in, and the
  // one-pass schedule where it applies) with the default merge tile first,
  // then the merge tiles with the best of those
  struct Sched {
    uint32_t handler, fanin;
  };
  std::vector<Sched> scheds;
  for (uint32_t F : {2u, 4u, 8u, 16u}) {
    if (F > 2 && F / 2 >= P) break;
    scheds.push_back(Sched{LBSORT_HANDLER_PASSES, F});
  }
  const bool one_ok = P >= 2 && P <= 64 && total_n <= (1ull << 32);
  uint32_t pow2P = 2;
  while (pow2P < P) pow2P *= 2;
  if (one_ok) scheds.push_back(Sched{LBSORT_HANDLER_ONE_PASS, pow2P});
  std::vector<uint32_t> rtiles = {4096, 8192};
  if (kb == 4) rtiles.push_back(16384);  // 32-bit keys also take tiles of 16384 keys
  const uint32_t mtiles[3] = {1024, 2048, 4096};
  void *kin = nullptr, *kout = nullptr, *kref = nullptr, *ws = nullptr;
  uint32_t *vin = nullptr, *vout = nullptr, *vref = nullptr;
  uint64_t *seg = nullptr, *offs = nullptr, *oref = nullptr;
  unsigned long long* diff = nullptr;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  hipStream_t st = nullptr;
  int rc = LBSORT_OK;
  size_t ws_need = 0;
  double best_ms = 1e30;
  uint32_t best_f = 0, best_t = 0, best_r = 0, best_h = 0, best_s = LBSORT_PRESORTED_DETECT;
  bool have_ref = false;
  lbsort_parts parts;
  memset(&parts, 0, sizeof parts);
  const uint64_t noffs = (uint64_t)B * (P + 1);
  auto measure = [&](uint32_t R, Sched h, uint32_t T, uint32_t S) -> int {
    lbsort_params prm = {P, 0, LBSORT_INV_COUNT, h.fanin, T, R, h.handler, S, 0};
    size_t wsb = ws_need;
    float times[5];
    for (int it = 0; it < 6; ++it) {
      if (hipEventRecord(e0, st) != hipSuccess) return LBSORT_ERR_HIP;
      int r2 = lbsort_sort_batch(key_type, val_type, kin, vin, kout, vout, seg, B, total_n, &prm, &parts, ws, &wsb, st);
      if (r2) return r2;
      if (hipEventRecord(e1, st) != hipSuccess || hipEventSynchronize(e1) != hipSuccess) return LBSORT_ERR_HIP;
      if (it > 0 && hipEventElapsedTime(&times[it - 1], e0, e1) != hipSuccess) return LBSORT_ERR_HIP;
    }
    int dev = lbsort_check(ws, st);
    if (dev) return dev;
    if (!have_ref) {
      if (hipMemcpyAsync(kref, kout, total_n * kb, hipMemcpyDeviceToDevice, st) != hipSuccess ||
          (hasv && hipMemcpyAsync(vref, vout, total_n * 4, hipMemcpyDeviceToDevice, st) != hipSuccess) ||
          hipMemcpyAsync(oref, offs, noffs * 8, hipMemcpyDeviceToDevice, st) != hipSuccess)
        return LBSORT_ERR_HIP;
      have_ref = true;
    } else {
      // every candidate must produce the same bytes
      unsigned long long nd = 0;
      if (hipMemsetAsync(diff, 0, sizeof(unsigned long long), st) != hipSuccess) return LBSORT_ERR_HIP;
      hipLaunchKernelGGL(k_diff, dim3(2048), dim3(256), 0, st, (const uint32_t*)kref, (const uint32_t*)kout,
                         total_n * kb / 4, diff);
      if (hasv)
        hipLaunchKernelGGL(k_diff, dim3(2048), dim3(256), 0, st, (const uint32_t*)vref, (const uint32_t*)vout, total_n,
                           diff);
      hipLaunchKernelGGL(k_diff, dim3(64), dim3(256), 0, st, (const uint32_t*)oref, (const uint32_t*)offs, noffs * 2,
                         diff);
      if (hipMemcpyAsync(&nd, diff, sizeof nd, hipMemcpyDeviceToHost, st) != hipSuccess ||
          hipStreamSynchronize(st) != hipSuccess)
        return LBSORT_ERR_HIP;
      if (nd) return LBSORT_ERR_DEVICE;
    }
    std::sort(times, times + 5);
    if (times[2] < best_ms) {
      best_ms = times[2];
      best_f = h.fanin;
      best_t = T;
      best_r = R;
      best_h = h.handler;
      best_s = S;
    }
    return LBSORT_OK;
  };
  for (uint32_t R : rtiles)
    for (Sched h : scheds)
      for (uint32_t T : mtiles) {
        if (h.handler == LBSORT_HANDLER_ONE_PASS && T < 2048) continue;
        lbsort_params prm = {P, 0, LBSORT_INV_COUNT, h.fanin, T, R, h.handler, 0, 0};
        size_t need = 0;
        parts.part_offsets = (uint64_t*)1;  // the size query reads no pointer
        rc = lbsort_sort_batch(key_type, val_type, nullptr, nullptr, nullptr, nullptr, (const uint64_t*)1, B, total_n,
                               &prm, &parts, nullptr, &need, nullptr);
        if (rc) goto done;
        ws_need = std::max(ws_need, need);
      }
  if (hipStreamCreate(&st) != hipSuccess || hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
    rc = LBSORT_ERR_HIP;
    goto done;
  }
  if (hipMalloc(&kout, total_n * kb) || hipMalloc(&kref, total_n * kb) || hipMalloc(&ws, ws_need) ||
      hipMalloc(&offs, noffs * 8) || hipMalloc(&oref, noffs * 8) || hipMalloc(&diff, sizeof(unsigned long long)) ||
      (hasv && (hipMalloc(&vout, total_n * 4) || hipMalloc(&vref, total_n * 4)))) {
    rc = LBSORT_ERR_OOM;
    goto done;
  }
  if (keys_in) {
    kin = (void*)keys_in;
    vin = (uint32_t*)vals_in;
  } else {
    if (hipMalloc(&kin, total_n * kb) || (val_type == LBSORT_VAL_U32 && hipMalloc(&vin, total_n * 4))) {
      rc = LBSORT_ERR_OOM;
      goto done;
    }
    hipLaunchKernelGGL(k_gen, dim3(4096), dim3(256), 0, st, kin, vin, total_n, kb == 8 ? 1 : 0,
                       (uint64_t)0x51ed270b27ull);
  }
  if (seg_offsets) {
    seg = (uint64_t*)seg_offsets;
  } else {
    // equal instances (the last one takes the remainder)
    std::vector<uint64_t> hseg(B + 1);
    for (uint32_t b = 0; b < B; ++b) hseg[b] = (uint64_t)b * (total_n / B);
    hseg[B] = total_n;
    if (hipMalloc(&seg, (B + 1) * 8) ||
        hipMemcpyAsync(seg, hseg.data(), (B + 1) * 8, hipMemcpyHostToDevice, st) != hipSuccess ||
        hipStreamSynchronize(st) != hipSuccess) {
      rc = LBSORT_ERR_HIP;
      goto done;
    }
  }
  parts.part_offsets = offs;
  for (uint32_t R : rtiles)
    for (Sched h : scheds)
      if ((rc = measure(R, h, h.handler == LBSORT_HANDLER_ONE_PASS ? 4096 : 2048, LBSORT_PRESORTED_DETECT)) !=
          LBSORT_OK)
        goto done;
  {
    const uint32_t R = best_r, T0 = best_t;
    const Sched h = {best_h, best_f};
    for (uint32_t T : mtiles)
      if (T != T0 && !(h.handler == LBSORT_HANDLER_ONE_PASS && T < 2048) &&
          (rc = measure(R, h, T, LBSORT_PRESORTED_DETECT)) != LBSORT_OK)
        goto done;
  }
  {
    // the same settings without looking for presorted blocks
    const Sched h = {best_h, best_f};
    if ((rc = measure(best_r, h, best_t, LBSORT_PRESORTED_IGNORE)) != LBSORT_OK) goto done;
  }
  {
    std::lock_guard<std::mutex> lk(g_mu);
    upsert(Entry{arch, (uint32_t)kb, hasv ? 1u : 0u, size_class(total_n / B), B > 1 ? 1u : 0u, P, best_f, best_t,
                 best_r, best_h, best_s, best_ms});
    const char* path = (cache_path && *cache_path) ? cache_path : getenv("LBSORT_TUNE_CACHE");
    if (path && *path && write_file(path) != 0) rc = LBSORT_ERR_INVALID_ARG;
  }
  if (chosen) {
    lbsort_params c = {P, 0, LBSORT_INV_COUNT, best_f, best_t, best_r, best_h, best_s, 0};
    *chosen = c;
  }
done:
  if (st) hipStreamSynchronize(st);
  if (!keys_in) {
    hipFree(kin);
    hipFree(vin);
  }
  if (!seg_offsets) hipFree(seg);
  hipFree(kout);
  hipFree(kref);
  hipFree(vout);
  hipFree(vref);
  hipFree(ws);
  hipFree(offs);
  hipFree(oref);
  hipFree(diff);
  if (e0) hipEventDestroy(e0);
  if (e1) hipEventDestroy(e1);
  if (st) hipStreamDestroy(st);
  return rc;
}

// ----------------------------------------------------------------- profiling
namespace lbs {

struct ProfRec {
  const char* name;
  int a, b;
};
static bool g_prof_on = false;
static std::vector<hipEvent_t> g_events;
static std::vector<ProfRec> g_recs;
static size_t g_next_event = 0;

static int take_event() {
  if (g_next_event == g_events.size()) {
    hipEvent_t e;
    if (hipEventCreate(&e) != hipSuccess) return -1;
    g_events.push_back(e);
  }
  return (int)g_next_event++;
}

int prof_begin(hipStream_t s) {
  if (!g_prof_on) return -1;
  int a = take_event();
  if (a >= 0) hipEventRecord(g_events[a], s);
  return a;
}

void prof_end(int id, const char* name, hipStream_t s) {
  if (id < 0 || !g_prof_on) return;
  int b = take_event();
  if (b < 0) return;
  hipEventRecord(g_events[b], s);
  g_recs.push_back(ProfRec{name, id, b});
}

}  // namespace lbs

extern "C" int lbsort_profile_enable(int on) {
  lbs::g_prof_on = on != 0;
  return LBSORT_OK;
}

extern "C" int lbsort_profile_read(char* buf, size_t len) {
  using namespace lbs;
  // A size query (buf == NULL) leaves the records in place.
  std::vector<std::string> names;
  std::vector<double> ms;
  std::vector<int> cnt;
  for (auto& r : g_recs) {
    hipEventSynchronize(g_events[r.b]);
    float t = 0;
    hipEventElapsedTime(&t, g_events[r.a], g_events[r.b]);
    size_t i = 0;
    while (i < names.size() && names[i] != r.name) ++i;
    if (i == names.size()) {
      names.push_back(r.name);
      ms.push_back(0);
      cnt.push_back(0);
    }
    ms[i] += t;
    cnt[i] += 1;
  }
  std::string out;
  char line[256];
  for (size_t i = 0; i < names.size(); ++i) {
    snprintf(line, sizeof line, "%s %d %.6f\n", names[i].c_str(), cnt[i], ms[i]);
    out += line;
  }
  if (buf && len) {
    size_t n = out.size() < len - 1 ? out.size() : len - 1;
    memcpy(buf, out.data(), n);
    buf[n] = 0;
    g_recs.clear();
    g_next_event = 0;
  }
  return (int)out.size();
}
