// Tuned tile shapes and thresholds: the table the project's autotuner writes (tuning.txt next to the
// library, or the file named by HQ_TUNING), read once at first use, and its C ABI.
#include <dlfcn.h>

#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <string>

#include "../../include/hq.h"
#include "kernels.h"
#include "predictor.h"

namespace hq {
namespace {
std::string g_source = "defaults";

std::string table_path() {
  if (const char* e = std::getenv("HQ_TUNING")) return e;
  Dl_info di;
  if (dladdr(reinterpret_cast<const void*>(&tuning), &di) && di.dli_fname) {
    std::string f = di.dli_fname;
    const size_t slash = f.rfind('/');
    return (slash == std::string::npos ? std::string(".") : f.substr(0, slash)) + "/tuning.txt";
  }
  return "tuning.txt";
}

// "key value" lines; '#' starts a comment; unknown keys are ignored.  An entry that leaves the
// table out of range discards the whole file (defaults stay).
void load(Tuning& t) {
  const std::string path = table_path();
  FILE* f = std::fopen(path.c_str(), "r");
  if (!f) return;
  Tuning n = t;
  char line[512];
  while (std::fgets(line, sizeof line, f)) {
    char key[128];
    long v = 0;
    if (line[0] == '#' || std::sscanf(line, "%127s %ld", key, &v) != 2) continue;
    if (!std::strcmp(key, "qr_tile_rows")) n.qr_tile_rows = (int)v;
    else if (!std::strcmp(key, "split_min_k")) n.split_min_k = (int)v;
    else if (!std::strcmp(key, "split_chunk")) n.split_chunk = (int)v;
    else if (!std::strcmp(key, "split_max")) n.split_max = (int)v;
    else if (!std::strcmp(key, "schur_keep")) n.schur_keep = (int)v;
    else if (!std::strcmp(key, "gemm_small_tiles")) n.gemm_small_tiles = (int)v;
  }
  std::fclose(f);
  if (n.valid()) {
    t = n;
    g_source = path;
  }
}
}  // namespace

Tuning& tuning() {
  static Tuning t;
  static std::once_flag once;
  std::call_once(once, [] { load(t); });
  return t;
}
}  // namespace hq

extern "C" hq_status hq_tuning_get(hq_tuning* out) {
  if (!out) {
    hq::set_last_error("out is NULL");
    return HQ_ERR_ARG;
  }
  const hq::Tuning& t = hq::tuning();
  out->qr_tile_rows = t.qr_tile_rows;
  out->split_min_k = t.split_min_k;
  out->split_chunk = t.split_chunk;
  out->split_max = t.split_max;
  out->schur_keep = t.schur_keep;
  out->gemm_small_tiles = t.gemm_small_tiles;
  return HQ_OK;
}

extern "C" hq_status hq_tuning_set(const hq_tuning* in) {
  if (!in) {
    hq::set_last_error("tuning is NULL");
    return HQ_ERR_ARG;
  }
  hq::Tuning n;
  n.qr_tile_rows = in->qr_tile_rows;
  n.split_min_k = in->split_min_k;
  n.split_chunk = in->split_chunk;
  n.split_max = in->split_max;
  n.schur_keep = in->schur_keep;
  n.gemm_small_tiles = in->gemm_small_tiles;
  if (!n.valid()) {
    hq::set_last_error("tuning values out of range");
    return HQ_ERR_ARG;
  }
  hq::tuning() = n;
  hq::g_source = "hq_tuning_set";
  return HQ_OK;
}

extern "C" const char* hq_tuning_source(void) {
  (void)hq::tuning();
  return hq::g_source.c_str();
}
