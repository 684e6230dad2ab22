// Persisted choices of the int8 autotuner (host code only).
//
// With PINV_AUTOTUNE_CACHE naming a file, pinv_autotune_int8 first looks for
// an entry of the same device kind and problem there and, if one is found,
// takes its variant without timing; otherwise it times the variants and
// appends the choice.  One entry per line, fields separated by blanks:
//
//   int8 <arch> <compute units> <unknowns> <S> <SR> <padded rhs> <variant> <ms>
//
// A later line overrides an earlier one with the same key; lines that do not
// parse (other tools' notes, a line cut short) are skipped.  The file is only
// appended to, one whole line per write, so concurrent tuners at worst both
// time and both append.

#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>

#include "common.h"

namespace {

std::mutex g_cache_mu;

}  // namespace

std::string tune_device_key(int device) {
  hipDeviceProp_t p{};
  if (hipGetDeviceProperties(&p, device) != hipSuccess) return std::string();
  std::string arch(p.gcnArchName);
  for (char& c : arch)
    if (c == ' ' || c == '\t' || c == '\n') c = '_';
  if (arch.empty()) return std::string();
  return arch + " " + std::to_string(p.multiProcessorCount);
}

bool tune_cache_lookup(const char* path, const std::string& dkey, int n, int S, int SR, int Rpad, int nvariants,
                       int* variant, double* ms) {
  if (!path || !*path || dkey.empty()) return false;
  std::lock_guard<std::mutex> lk(g_cache_mu);
  FILE* f = std::fopen(path, "r");
  if (!f) return false;
  bool found = false;
  char line[512];
  while (std::fgets(line, sizeof line, f)) {
    if (!std::strchr(line, '\n') && !std::feof(f)) {
      // longer than any entry: skip the rest of it
      int c;
      while ((c = std::fgetc(f)) != EOF && c != '\n') {
      }
      continue;
    }
    char kind[16], arch[256];
    int cus, ln, lS, lSR, lR, v;
    double t;
    if (std::sscanf(line, "%15s %255s %d %d %d %d %d %d %lf", kind, arch, &cus, &ln, &lS, &lSR, &lR, &v, &t) != 9)
      continue;
    if (std::strcmp(kind, "int8") != 0 || v < 0 || v >= nvariants || !(t > 0.0)) continue;
    if (dkey != std::string(arch) + " " + std::to_string(cus)) continue;
    if (ln != n || lS != S || lSR != SR || lR != Rpad) continue;
    *variant = v;
    *ms = t;
    found = true;
  }
  std::fclose(f);
  return found;
}

void tune_cache_store(const char* path, const std::string& dkey, int n, int S, int SR, int Rpad, int variant,
                      double ms) {
  if (!path || !*path || dkey.empty()) return;
  char line[512];
  const int len = std::snprintf(line, sizeof line, "int8 %s %d %d %d %d %d %.6f\n", dkey.c_str(), n, S, SR, Rpad,
                                variant, ms);
  if (len <= 0 || len >= (int)sizeof line) return;
  std::lock_guard<std::mutex> lk(g_cache_mu);
  FILE* f = std::fopen(path, "a");
  if (!f) {
    pinv_log("autotune cache: cannot append to %s", path);
    return;
  }
  std::fputs(line, f);
  std::fclose(f);
}
