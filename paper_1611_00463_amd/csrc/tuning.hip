// Autotuner for the handler merge: picks the fan-in F and the merge tile per
// shape by timing every candidate on the device, checks that every candidate
// produced the same bytes, and keeps the winner in an in-process table that
// can be saved to / loaded from a small JSON file.
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
  int key_type, val_type;
  uint32_t size_log2, batched, P, fanin, merge_tile;
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

static int parse_file(const char* path, std::vector<Entry>& out) {
  FILE* f = fopen(path, "r");
  if (!f) return -1;
  std::string s;
  char buf[4096];
  size_t r;
  while ((r = fread(buf, 1, sizeof buf, f)) > 0) s.append(buf, r);
  fclose(f);
  // One object per entry: {"key": .., "val": .., "size_log2": .., "batched": .., "P": .., "fanin": .., "merge_tile": .., "ms": ..}
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
    double k, vt, sl, b, P, F, T, ms = 0;
    if (num("key", k) && num("val", vt) && num("size_log2", sl) && num("batched", b) && num("P", P) &&
        num("fanin", F) && num("merge_tile", T)) {
      num("ms", ms);
      out.push_back(Entry{(int)k, (int)vt, (uint32_t)sl, (uint32_t)b, (uint32_t)P, (uint32_t)F, (uint32_t)T, ms});
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
            "  {\"key\": %d, \"val\": %d, \"size_log2\": %u, \"batched\": %u, \"P\": %u, \"fanin\": %u, "
            "\"merge_tile\": %u, \"ms\": %.4f}%s\n",
            e.key_type, e.val_type, e.size_log2, e.batched, e.P, e.fanin, e.merge_tile, e.ms,
            i + 1 < g_table.size() ? "," : "");
  }
  fprintf(f, "]}\n");
  fclose(f);
  return 0;
}

static void upsert(const Entry& e) {
  for (auto& x : g_table)
    if (x.key_type == e.key_type && x.val_type == e.val_type && x.size_log2 == e.size_log2 &&
        x.batched == e.batched && x.P == e.P) {
      x = e;
      return;
    }
  g_table.push_back(e);
}

Tuned tuning_lookup(int key_type, int val_type, uint64_t n, uint32_t B, uint32_t P) {
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
  const uint32_t sc = size_class(n);
  const uint32_t batched = B > 1 ? 1 : 0;
  const Entry* best = nullptr;
  for (auto& e : g_table) {
    if (e.key_type != key_type || e.val_type != val_type || e.batched != batched || e.P != P) continue;
    if (!best || (uint32_t)abs((int)e.size_log2 - (int)sc) < (uint32_t)abs((int)best->size_log2 - (int)sc)) best = &e;
  }
  Tuned t = {0, 0};
  if (best && (uint32_t)abs((int)best->size_log2 - (int)sc) <= 2) {
    t.fanin = best->fanin;
    t.merge_tile = best->merge_tile;
  }
  return t;
}

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

extern "C" int lbsort_autotune(int key_type, int val_type, uint64_t n, uint32_t B, uint32_t P, const char* cache_path,
                               uint32_t* fanin_out, uint32_t* tile_out) {
  if ((key_type != LBSORT_U32 && key_type != LBSORT_U64) || (val_type != LBSORT_NOVAL && val_type != LBSORT_VAL_U32) ||
      n == 0 || B == 0 || P < 1 || P > LBSORT_MAX_P)
    return LBSORT_ERR_INVALID_ARG;
  const uint64_t kb = key_type == LBSORT_U64 ? 8 : 4;
  const uint64_t total = n * B;
  void *kin = nullptr, *kout = nullptr, *ref = nullptr, *ws = nullptr, *parts_mem = nullptr;
  uint32_t *vin = nullptr, *vout = nullptr;
  uint64_t* seg = nullptr;
  int rc = LBSORT_OK;
  std::vector<uint64_t> hseg(B + 1);
  for (uint32_t b = 0; b <= B; ++b) hseg[b] = (uint64_t)b * n;
  std::vector<uint32_t> fans;
  for (uint32_t F : {2u, 4u, 8u, 16u}) {
    if (F > 2 && F / 2 >= P) break;
    fans.push_back(F);
  }
  const uint32_t tiles[3] = {1024, 2048, 4096};
  size_t ws_need = 0;
  double best_ms = 1e30;
  uint32_t best_f = 0, best_t = 0;
  hipEvent_t e0, e1;
  hipEventCreate(&e0);
  hipEventCreate(&e1);
  lbsort_parts parts;
  memset(&parts, 0, sizeof parts);
  for (uint32_t F : fans)
    for (uint32_t T : tiles) {
      lbsort_params prm = {P, 0, LBSORT_INV_COUNT, F, T, 0};
      size_t need = 0;
      int r2 = lbsort_sort_batch(key_type, val_type, nullptr, nullptr, nullptr, nullptr, (const uint64_t*)1, B, total,
                                 &prm, &parts, nullptr, &need, nullptr);
      if (r2) return r2;
      ws_need = std::max(ws_need, need);
    }
  if (hipMalloc(&kin, total * kb) || hipMalloc(&kout, total * kb) || hipMalloc(&ref, total * kb) ||
      hipMalloc(&ws, ws_need) || hipMalloc(&seg, (B + 1) * 8) || hipMalloc(&parts_mem, (uint64_t)B * (P + 1) * 8) ||
      (val_type && (hipMalloc(&vin, total * 4) || hipMalloc(&vout, total * 4)))) {
    rc = LBSORT_ERR_OOM;
    goto done;
  }
  hipMemcpy(seg, hseg.data(), (B + 1) * 8, hipMemcpyHostToDevice);
  hipLaunchKernelGGL(k_gen, dim3(4096), dim3(256), 0, nullptr, kin, vin, total, key_type == LBSORT_U64 ? 1 : 0,
                     (uint64_t)0x51ed270b27ull);
  parts.part_offsets = (uint64_t*)parts_mem;
  {
    bool have_ref = false;
    for (uint32_t F : fans)
      for (uint32_t T : tiles) {
        lbsort_params prm = {P, 0, LBSORT_INV_COUNT, F, T, 0};
        size_t wsb = ws_need;
        float times[5];
        for (int it = 0; it < 6; ++it) {
          hipEventRecord(e0, nullptr);
          int r2 = lbsort_sort_batch(key_type, val_type, kin, vin, kout, vout, seg, B, total, &prm, &parts, ws, &wsb,
                                     nullptr);
          hipEventRecord(e1, nullptr);
          if (r2) {
            rc = r2;
            goto done;
          }
          hipEventSynchronize(e1);
          if (it > 0) hipEventElapsedTime(&times[it - 1], e0, e1);
        }
        int dev = lbsort_check(ws, nullptr);
        if (dev) {
          rc = dev;
          goto done;
        }
        std::sort(times, times + 5);
        if (!have_ref) {
          hipMemcpy(ref, kout, total * kb, hipMemcpyDeviceToDevice);
          have_ref = true;
        } else {
          std::vector<char> a(total * kb), b(total * kb);
          hipMemcpy(a.data(), ref, total * kb, hipMemcpyDeviceToHost);
          hipMemcpy(b.data(), kout, total * kb, hipMemcpyDeviceToHost);
          if (memcmp(a.data(), b.data(), total * kb) != 0) {
            rc = LBSORT_ERR_DEVICE;
            goto done;
          }
        }
        if (times[2] < best_ms) {
          best_ms = times[2];
          best_f = F;
          best_t = T;
        }
      }
  }
  {
    std::lock_guard<std::mutex> lk(g_mu);
    upsert(Entry{key_type, val_type, size_class(n), B > 1 ? 1u : 0u, P, best_f, best_t, best_ms});
    if (cache_path && *cache_path) write_file(cache_path);
    else {
      const char* env = getenv("LBSORT_TUNE_CACHE");
      if (env && *env) write_file(env);
    }
  }
  if (fanin_out) *fanin_out = best_f;
  if (tile_out) *tile_out = best_t;
done:
  hipDeviceSynchronize();
  hipFree(kin);
  hipFree(kout);
  hipFree(ref);
  hipFree(ws);
  hipFree(seg);
  hipFree(parts_mem);
  if (vin) hipFree(vin);
  if (vout) hipFree(vout);
  hipEventDestroy(e0);
  hipEventDestroy(e1);
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
