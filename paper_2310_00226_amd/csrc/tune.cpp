// Tuning cache of the kernel choices (tile shapes, tile orders) that the library
// picks by timing: process-wide, keyed by device architecture, kernel and the
// geometry of the pass, and kept across processes in a JSON file named by the
// environment variable SEM_TUNE_CACHE (read on first use, rewritten after every
// new entry; no file when the variable is unset).  File format:
//   {"version": 1, "entries": {"<key>": <int>, ...}}
#include "tune.h"

#include <cstdio>
#include <cstdlib>
#include <fstream>
#include <map>
#include <mutex>
#include <sstream>
#include <string>

#include <unistd.h>

namespace semfd {
namespace {

std::mutex g_mutex;
bool g_loaded = false;
std::map<std::string, int> g_entries;
int g_hits = 0, g_misses = 0;

const char* cache_path() {
  const char* p = std::getenv("SEM_TUNE_CACHE");
  return p && *p ? p : nullptr;
}

// Minimal reader of the flat format written by save(): "key": integer pairs
// inside the "entries" object; anything unreadable leaves the cache empty.
void load_locked() {
  g_loaded = true;
  const char* path = cache_path();
  if (!path) return;
  std::ifstream in(path);
  if (!in) return;
  std::stringstream ss;
  ss << in.rdbuf();
  const std::string text = ss.str();
  const size_t ent = text.find("\"entries\"");
  if (ent == std::string::npos) return;
  size_t i = text.find('{', ent);
  if (i == std::string::npos) return;
  std::map<std::string, int> got;
  while (true) {
    const size_t q0 = text.find('"', i + 1);
    const size_t close = text.find('}', i + 1);
    if (q0 == std::string::npos || (close != std::string::npos && close < q0)) break;
    const size_t q1 = text.find('"', q0 + 1);
    if (q1 == std::string::npos) return;
    const size_t colon = text.find(':', q1);
    if (colon == std::string::npos) return;
    char* end = nullptr;
    const long v = std::strtol(text.c_str() + colon + 1, &end, 10);
    if (end == text.c_str() + colon + 1) return;
    got[text.substr(q0 + 1, q1 - q0 - 1)] = (int)v;
    i = (size_t)(end - text.c_str());
  }
  g_entries.swap(got);
}

void save_locked() {
  const char* path = cache_path();
  if (!path) return;
  // a temporary file of this process, renamed over the cache in one step, so a
  // reader (or another process saving at the same time) never sees a partial file
  const std::string tmp = std::string(path) + ".tmp." + std::to_string((long)getpid());
  {
    std::ofstream out(tmp, std::ios::trunc);
    if (!out) return;
    out << "{\"version\": 1, \"entries\": {";
    bool first = true;
    for (const auto& kv : g_entries) {
      out << (first ? "\n  " : ",\n  ") << '"' << kv.first << "\": " << kv.second;
      first = false;
    }
    out << "\n}}\n";
  }
  std::rename(tmp.c_str(), path);
}

}  // namespace

bool tune_lookup(const std::string& key, int* value) {
  std::lock_guard<std::mutex> lock(g_mutex);
  if (!g_loaded) load_locked();
  auto it = g_entries.find(key);
  if (it == g_entries.end()) {
    ++g_misses;
    return false;
  }
  ++g_hits;
  *value = it->second;
  return true;
}

void tune_store(const std::string& key, int value) {
  std::lock_guard<std::mutex> lock(g_mutex);
  if (!g_loaded) load_locked();
  g_entries[key] = value;
  save_locked();
}

void tune_counts(int* hits, int* misses) {
  std::lock_guard<std::mutex> lock(g_mutex);
  *hits = g_hits;
  *misses = g_misses;
}

int tune_size() {
  std::lock_guard<std::mutex> lock(g_mutex);
  if (!g_loaded) load_locked();
  return (int)g_entries.size();
}

int tune_bucket(long v) {
  int b = 0;
  while (v > 1) {
    v >>= 1;
    ++b;
  }
  return b;
}

}  // namespace semfd
