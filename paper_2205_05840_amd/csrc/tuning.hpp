// Launch shapes measured by the autotuner (paper_2205_05840_amd/tune.py), looked up by the
// launchers before their cost models.  A table is valid only for the kernel sources it was
// measured on: its key must equal source_key(), a hash of those sources taken at build time.
#pragma once

#include <string>

namespace ndmg {

enum TuneKind : int {
  kTuneStencil = 0,   // plane-marching operator kernel: p0 = variant index, p1 = planes per workgroup
  kTunePatch = 1,     // vertex patch products: p0 = groups per wave (interior segment),
                      // p1 = groups per wave (segments on the faces and edges of the box)
  kTunePatchAddr = 2, // addressing of the smoother's condensation and patch products: p0 =
                      // 64 for 64-bit addresses, 32 for 32-bit buffer offsets where the
                      // vectors allow them (p1 unused)
};

// Pairs per launch, in classes: 1, 2-3, 4-15, 16-63, 64 and more.
int tune_count_class(int count);

// The tuned shape for (kind, n, element bytes, mode, pairs per launch), if the table holds one.
bool tune_lookup(int kind, int n, int elem, int mode, int count, int* p0, int* p1);

// While set (non-negative), the stencil launcher uses this shape whatever the table or the
// cost model say (the tuner's timing calls); per thread.
void tune_force_stencil(int variant, int kz);

bool tune_forced_stencil(int* variant, int* kz);

const char* source_key();

// Table text: "key <source key>", then lines "<stencil|patch|patchaddr> <n> <fp32|fp64>
// <mode> <pair class> <p0> <p1>"; '#' starts a comment.
bool tune_load(const std::string& path, std::string* err);
bool tune_set_line(const std::string& line, std::string* err);
void tune_clear();

}  // namespace ndmg
