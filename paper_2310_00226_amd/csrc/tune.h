// Tuning cache of kernel choices made by timing (tune.cpp).
#pragma once
#include <string>

namespace semfd {
// Cached choice for key (false: not tuned yet).  Keys start with the device
// architecture (gcnArchName) and name the kernel and the pass geometry.
bool tune_lookup(const std::string& key, int* value);
// Record a choice (and rewrite the file named by SEM_TUNE_CACHE, if set).
void tune_store(const std::string& key, int value);
// Lookups answered from the cache / not found, since the process started.
void tune_counts(int* hits, int* misses);
// Entries held (after reading the file on first use).
int tune_size();
// floor(log2(v)) for v >= 1 (0 for v <= 1): the size buckets of the keys.
int tune_bucket(long v);
}  // namespace semfd
