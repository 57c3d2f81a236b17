// Schedule parameters of the batched form and their JSON tune cache (host
// code only).  The cache is a file the caller names, so every entry read
// back is checked against the ranges the schedule supports before it is
// used; an entry outside them is ignored and the batch is tuned again.
#pragma once

#include <cmath>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

namespace fockx {

constexpr int kBatchSlots = 6;   // pair buffers the persistent schedule allocates
constexpr int kBatchStages = 4;  // P1, P2, P3, MAC: tiles in flight at once

struct BatchParams {
  int tile = 16;             // pair tile edge: 8 or 16
  int slots = kBatchSlots;   // pair buffers in flight, kBatchStages .. kBatchSlots
  int units_per_ticket = 8;  // work units a block takes per ticket (>= 1)
  int blocks_per_cu = 1;     // persistent blocks per CU (selects the register budget)
  double ms = 0.0;           // measured replay time when tuned
  // 0: one persistent kernel runs every stage of every system; 1: the graph
  // holds each system's own schedule of per-shape kernels
  int mode = 0;
  // mode 1: independent graph branches the systems are split over (1: one
  // after another)
  int branches = 1;
};

constexpr int kBatchMaxBranches = 4;

// Ranges the persistent schedule is built for.  slots below kBatchStages
// would make a pair tile wait on a later tile of the same buffer ring (a
// dependency on work not yet handed out); above kBatchSlots it would index
// past the buffer table; a tile edge above 16 overruns the buffers, sized
// for 16 x 16 pairs; no units per ticket means no work is ever taken.
inline bool batch_params_valid(const BatchParams& p) {
  return (p.tile == 8 || p.tile == 16) && p.slots >= kBatchStages && p.slots <= kBatchSlots &&
         p.units_per_ticket >= 1 && p.units_per_ticket <= (1 << 20) && p.blocks_per_cu >= 1 &&
         p.blocks_per_cu <= 8 && (p.mode == 0 || p.mode == 1) && p.branches >= 1 &&
         p.branches <= kBatchMaxBranches && std::isfinite(p.ms) && p.ms >= 0.0;
}

// Entry for `key` in the cache file at `path` (the last one if repeated).
// Returns false when there is none, or when it is malformed or out of range.
inline bool tune_cache_lookup(const std::string& path, const std::string& key, BatchParams* out) {
  if (path.empty() || key.empty()) return false;
  FILE* f = std::fopen(path.c_str(), "r");
  if (!f) return false;
  char line[4096];
  bool found = false;
  const std::string pat = "\"" + key + "\": {";
  while (std::fgets(line, sizeof line, f)) {
    const char* at = std::strstr(line, pat.c_str());
    if (!at) continue;
    BatchParams p;
    // entries written before the mode field existed describe the persistent
    // kernel, those before the branches field one branch
    const int got = std::sscanf(at + pat.size(),
                                " \"tile\": %d, \"slots\": %d, \"units_per_ticket\": %d, \"blocks_per_cu\": %d, "
                                "\"ms\": %lf, \"mode\": %d, \"branches\": %d",
                                &p.tile, &p.slots, &p.units_per_ticket, &p.blocks_per_cu, &p.ms, &p.mode, &p.branches);
    if (got >= 5 && batch_params_valid(p)) {
      *out = p;
      found = true;
    } else {
      found = false;  // a later malformed entry for the key discards an earlier one
    }
  }
  std::fclose(f);
  return found;
}

// Writes (or replaces) the entry for `key`, keeping the file's other entries.
inline void tune_cache_store(const std::string& path, const std::string& key, const BatchParams& p) {
  if (path.empty() || !batch_params_valid(p)) return;
  std::vector<std::string> keep;
  if (FILE* f = std::fopen(path.c_str(), "r")) {
    char line[4096];
    const std::string pat = "\"" + key + "\": {";
    while (std::fgets(line, sizeof line, f)) {
      std::string l(line);
      if (l.find("\": {") != std::string::npos && l.find(pat) == std::string::npos) {
        while (!l.empty() && (l.back() == '\n' || l.back() == ',')) l.pop_back();
        keep.push_back(l);
      }
    }
    std::fclose(f);
  }
  char buf[512];
  std::snprintf(buf, sizeof buf,
                "\"%s\": {\"tile\": %d, \"slots\": %d, \"units_per_ticket\": %d, \"blocks_per_cu\": %d, \"ms\": %.4f, "
                "\"mode\": %d, \"branches\": %d}",
                key.c_str(), p.tile, p.slots, p.units_per_ticket, p.blocks_per_cu, p.ms, p.mode, p.branches);
  keep.push_back(buf);
  const std::string tmp = path + ".tmp";
  FILE* f = std::fopen(tmp.c_str(), "w");
  if (!f) return;
  std::fprintf(f, "{\n");
  for (size_t k = 0; k < keep.size(); ++k) std::fprintf(f, "%s%s\n", keep[k].c_str(), k + 1 < keep.size() ? "," : "");
  std::fprintf(f, "}\n");
  std::fclose(f);
  std::rename(tmp.c_str(), path.c_str());
}

}  // namespace fockx
