// tune.cpp -- autotuner table (see tune.hpp).
#include "tune.hpp"

#include <algorithm>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>

#include "runtime.hpp"

namespace lrsp {
namespace tune {

namespace {
std::mutex g_mu;
std::map<std::string, Choice> g_table;

int round_pow2(int v) {
  int p = 1;
  while (p < v) p <<= 1;
  return p;
}
}  // namespace

std::string key(bool batched, int max_m, int nitems, int ncolours) {
  char buf[96];
  std::snprintf(buf, sizeof(buf), "%s/m%d/n%d/c%d", batched ? "batch" : "single",
                ((max_m + 31) / 32) * 32, round_pow2(std::max(1, nitems)), ncolours);
  return buf;
}

bool lookup(const std::string& k, Choice* c) {
  std::lock_guard<std::mutex> g(g_mu);
  auto it = g_table.find(k);
  if (it == g_table.end()) return false;
  *c = it->second;
  return true;
}

void store(const std::string& k, const Choice& c) {
  std::lock_guard<std::mutex> g(g_mu);
  g_table[k] = c;
}

int entries() {
  std::lock_guard<std::mutex> g(g_mu);
  return (int)g_table.size();
}

void clear() {
  std::lock_guard<std::mutex> g(g_mu);
  g_table.clear();
}

// {"version": 1, "entries": [{"key": "...", "sched": s, "grid_cap": g, "tile": t, "ms": ms}, ...]}
lrsp_status save(const char* path) {
  if (!path) return rt::fail(LRSP_ERR_ARG, "null path");
  std::lock_guard<std::mutex> g(g_mu);
  FILE* f = std::fopen(path, "w");
  if (!f) return rt::fail(LRSP_ERR_ARG, std::string("cannot write ") + path);
  std::fprintf(f, "{\"version\": 1, \"entries\": [");
  bool first = true;
  for (auto& kv : g_table) {
    std::fprintf(f, "%s\n  {\"key\": \"%s\", \"sched\": %d, \"grid_cap\": %d, \"tile\": %d, \"ms\": %.6g}",
                 first ? "" : ",", kv.first.c_str(), kv.second.sched, kv.second.grid_cap, kv.second.tile,
                 kv.second.ms);
    first = false;
  }
  std::fprintf(f, "\n]}\n");
  std::fclose(f);
  return LRSP_OK;
}

// Reads files written by save(): every object with "key", "sched",
// "grid_cap" and "ms" fields becomes an entry.
lrsp_status load(const char* path) {
  if (!path) return rt::fail(LRSP_ERR_ARG, "null path");
  FILE* f = std::fopen(path, "r");
  if (!f) return rt::fail(LRSP_ERR_ARG, std::string("cannot read ") + path);
  std::string text;
  char buf[4096];
  size_t n;
  while ((n = std::fread(buf, 1, sizeof(buf), f)) > 0) text.append(buf, n);
  std::fclose(f);
  std::map<std::string, Choice> parsed;
  size_t pos = 0;
  while ((pos = text.find("\"key\"", pos)) != std::string::npos) {
    const size_t q0 = text.find('"', text.find(':', pos) + 1);
    const size_t q1 = q0 == std::string::npos ? q0 : text.find('"', q0 + 1);
    const size_t end = q1 == std::string::npos ? q1 : text.find('}', q1);
    if (end == std::string::npos) return rt::fail(LRSP_ERR_ARG, "malformed autotune file");
    const std::string k = text.substr(q0 + 1, q1 - q0 - 1);
    const std::string body = text.substr(q1, end - q1);
    Choice c;
    auto field = [&](const char* name, double* v) {
      const size_t p = body.find(name);
      if (p == std::string::npos) return false;
      const size_t c0 = body.find(':', p);
      return c0 != std::string::npos && std::sscanf(body.c_str() + c0 + 1, "%lf", v) == 1;
    };
    double s = 0, g = 0, ms = 0;
    if (!field("\"sched\"", &s) || !field("\"grid_cap\"", &g) || !field("\"ms\"", &ms))
      return rt::fail(LRSP_ERR_ARG, "malformed autotune entry " + k);
    if (s < 0 || s > 2) return rt::fail(LRSP_ERR_ARG, "invalid schedule in autotune entry " + k);
    double t = 0;  // optional (files without tiles: the default tile)
    if (field("\"tile\"", &t) && (t < 0 || t > 1))
      return rt::fail(LRSP_ERR_ARG, "invalid tile in autotune entry " + k);
    c.sched = (int)s;
    c.grid_cap = (int)g;
    c.tile = (int)t;
    c.ms = ms;
    parsed[k] = c;
    pos = end;
  }
  std::lock_guard<std::mutex> g(g_mu);
  for (auto& kv : parsed) g_table[kv.first] = kv.second;
  return LRSP_OK;
}

}  // namespace tune
}  // namespace lrsp
