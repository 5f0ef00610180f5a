// zmc_tune.hip -- the tile-shape table that the batched planner reads.
//
// The table is written by the project's autotuner (paper_1910_01965_amd/
// autotune.py), which times candidate tile shapes per kernel variant on the
// GPU.  It is looked up in $ZMC_TUNE_TABLE, else in tune_table.txt next to
// libzmc.so; variants missing from it take the built-in defaults below.
// Format: one variant per line, `family precision N pm_groups sm_groups
// pm_min_points`, '#' starts a comment.
#include <dlfcn.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <mutex>
#include <string>

#include "zmc.h"
#include "zmc_device.hpp"
#include "zmc_internal.hpp"

namespace zmc {
namespace {

constexpr int kFamilies = 5, kPrecisions = 2, kDims = kMaxDims;

struct Table {
  TuneEntry e[kFamilies][kPrecisions][kDims + 1];
  bool set[kFamilies][kPrecisions][kDims + 1];
  std::string source = "built-in defaults";
};

Table g_table;
std::once_flag g_once;

int family_id(const char* s) {
  static const char* names[kFamilies] = {"sin_sum", "gauss", "cosexp", "const", "linear"};
  for (int i = 0; i < kFamilies; ++i)
    if (strcmp(s, names[i]) == 0) return i;
  return -1;
}

int precision_id(const char* s) {
  if (strcmp(s, "fp64") == 0) return ZMC_FP64;
  if (strcmp(s, "fp32") == 0) return ZMC_FP32_MERGE64;
  return -1;
}

std::string table_path() {
  const char* env = getenv("ZMC_TUNE_TABLE");
  if (env && *env) return env;
  Dl_info info;
  if (dladdr((void*)&zmc_version, &info) && info.dli_fname) {
    std::string p(info.dli_fname);
    const size_t slash = p.rfind('/');
    return (slash == std::string::npos ? std::string(".") : p.substr(0, slash)) + "/tune_table.txt";
  }
  return "tune_table.txt";
}

void load() {
  memset(g_table.set, 0, sizeof(g_table.set));
  const std::string path = table_path();
  FILE* fh = fopen(path.c_str(), "r");
  if (!fh) {
    zmc::log(1, "tune table %s not found: built-in tile shapes", path.c_str());
    return;
  }
  char line[512];
  int rows = 0;
  while (fgets(line, sizeof(line), fh)) {
    char* hash = strchr(line, '#');
    if (hash) *hash = '\0';
    char fam[32], prec[16];
    int N = 0;
    long long pm = 0, sm = 0, pmin = 0;
    if (sscanf(line, "%31s %15s %d %lld %lld %lld", fam, prec, &N, &pm, &sm, &pmin) != 6) continue;
    const int f = family_id(fam), pr = precision_id(prec);
    if (f < 0 || pr < 0 || N < 1 || N > kDims || pm < 1 || sm < 1 || pmin < 1) continue;
    g_table.e[f][pr][N] = TuneEntry{pm, sm, pmin};
    g_table.set[f][pr][N] = true;
    ++rows;
  }
  fclose(fh);
  if (rows > 0) g_table.source = path;
  zmc::log(1, "tune table %s: %d rows", path.c_str(), rows);
}

}  // namespace

// Built-in defaults: a point-major tile of 256 lanes x 1024 groups (4096
// samples per lane) lasts about 2 ms at full occupancy, short enough for a
// small tail and long enough that per-tile setup is negligible; sample-major
// tiles take 16384 groups (64 per lane of a 256-thread block).
TuneEntry tune_lookup(int family, int precision, int N) {
  std::call_once(g_once, load);
  if (family >= 0 && family < kFamilies && precision >= 0 && precision < kPrecisions && N >= 1 &&
      N <= kDims && g_table.set[family][precision][N])
    return g_table.e[family][precision][N];
  return TuneEntry{1024, 16384, 128};
}

const char* tune_source() {
  std::call_once(g_once, load);
  return g_table.source.c_str();
}

}  // namespace zmc
