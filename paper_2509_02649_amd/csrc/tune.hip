// Launch-shape autotuner: a process-wide table of measured launch shapes, keyed by the GPU
// architecture and the problem shape, optionally persisted in a text file.
//
// Why: the grid search of Sec. 5 repeats one type-1 stage and many batched solves, and the
// best bin size, points per workgroup and launch widths depend on n, the number of channels
// and lambdas, and on the part.  Every candidate is a correct configuration of the same
// kernels (the results agree to rounding), so the tuner only picks the fastest.
//
// Table format (one entry per line; '#' starts a comment):
//     <key> = <name>=<int> <name>=<int> ... [ms=<float>]
//     e.g.  gfx950 t1 d=2 nf=512 w=7 nw=16 n=2^30 = mb=2 spread_pts=16384 sort_blk=512 sort_slice=65536 ms=75.3
// The file named by FK_AUTOTUNE_CACHE is read at the first lookup and every new measurement is
// appended to it.  FK_AUTOTUNE (or fk_options.autotune) selects the mode: tune at first use
// (default), built-in defaults only, or re-measure even when an entry exists.
#include "fk_internal.h"

#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <string>

namespace fk {

namespace {
std::mutex g_tune_mu;
std::map<std::string, std::string> g_table;   // key -> value text
bool g_file_loaded = false;

std::string trim(const std::string& s) {
  size_t a = s.find_first_not_of(" \t\r\n"), b = s.find_last_not_of(" \t\r\n");
  return a == std::string::npos ? std::string() : s.substr(a, b - a + 1);
}

// Parses "name=int name=int ..." (a trailing ms=<float> is kept as text); false on malformed input.
bool parse_values(const std::string& v, std::map<std::string, double>* out) {
  size_t i = 0;
  while (i < v.size()) {
    while (i < v.size() && (v[i] == ' ' || v[i] == '\t')) ++i;
    if (i >= v.size()) break;
    size_t j = v.find_first_of(" \t", i);
    if (j == std::string::npos) j = v.size();
    const std::string tok = v.substr(i, j - i);
    const size_t eq = tok.find('=');
    if (eq == std::string::npos || eq == 0 || eq + 1 >= tok.size()) return false;
    char* end = nullptr;
    const double x = std::strtod(tok.c_str() + eq + 1, &end);
    if (!end || *end != '\0' || !std::isfinite(x)) return false;
    (*out)[tok.substr(0, eq)] = x;
    i = j;
  }
  return !out->empty();
}

// Merge the lines of a cache file into the table; malformed lines are skipped.  Returns the number
// of entries taken.
int load_lines(FILE* f) {
  char buf[1024];
  int taken = 0;
  while (std::fgets(buf, sizeof(buf), f)) {
    std::string line(buf);
    const size_t hash = line.find('#');
    if (hash != std::string::npos) line = line.substr(0, hash);
    const size_t sep = line.find(" = ");
    if (sep == std::string::npos) continue;
    const std::string key = trim(line.substr(0, sep)), val = trim(line.substr(sep + 3));
    std::map<std::string, double> kv;
    if (key.empty() || !parse_values(val, &kv)) continue;
    g_table[key] = val;
    ++taken;
  }
  return taken;
}

void load_env_file_locked() {
  if (g_file_loaded) return;
  g_file_loaded = true;
  const char* path = std::getenv("FK_AUTOTUNE_CACHE");
  if (!path || !*path) return;
  FILE* f = std::fopen(path, "r");
  if (!f) return;
  load_lines(f);
  std::fclose(f);
}
}  // namespace

int tune_mode(const fk_ctx* ctx) {
  if (ctx && ctx->opt.autotune != 0) return ctx->opt.autotune;
  const char* e = std::getenv("FK_AUTOTUNE");
  if (!e) return kTuneAuto;
  if (!std::strcmp(e, "0") || !std::strcmp(e, "off")) return kTuneOff;
  if (!std::strcmp(e, "force") || !std::strcmp(e, "2")) return kTuneForce;
  return kTuneAuto;
}

std::string tune_arch(int device) {
  hipDeviceProp_t p;
  if (hipGetDeviceProperties(&p, device) != hipSuccess) return "gpu";
  std::string a(p.gcnArchName);
  const size_t c = a.find(':');
  return c == std::string::npos ? a : a.substr(0, c);
}

bool tune_lookup(const std::string& key, std::map<std::string, double>* values) {
  std::lock_guard<std::mutex> lk(g_tune_mu);
  load_env_file_locked();
  auto it = g_table.find(key);
  if (it == g_table.end()) return false;
  values->clear();
  return parse_values(it->second, values);
}

void tune_store(const std::string& key, const std::map<std::string, double>& values, double ms) {
  std::string v;
  for (const auto& kv : values) {
    char b[64];
    std::snprintf(b, sizeof(b), "%s%s=%lld", v.empty() ? "" : " ", kv.first.c_str(), (long long)kv.second);
    v += b;
  }
  char b[64];
  std::snprintf(b, sizeof(b), " ms=%.4f", ms);
  v += b;
  std::lock_guard<std::mutex> lk(g_tune_mu);
  load_env_file_locked();
  g_table[key] = v;
  const char* path = std::getenv("FK_AUTOTUNE_CACHE");
  if (path && *path) {
    FILE* f = std::fopen(path, "a");
    if (f) {
      std::fprintf(f, "%s = %s\n", key.c_str(), v.c_str());
      std::fclose(f);
    }
  }
}

}  // namespace fk

using namespace fk;

extern "C" fk_status fk_autotune_load(const char* path) {
  if (!path) return FK_EINVAL;
  FILE* f = std::fopen(path, "r");
  if (!f) return FK_EINVAL;
  std::lock_guard<std::mutex> lk(g_tune_mu);
  g_file_loaded = true;   // an explicit file takes the place of the environment's
  load_lines(f);
  std::fclose(f);
  return FK_OK;
}

extern "C" fk_status fk_autotune_table(char* buf, size_t cap, size_t* len) {
  std::string s;
  {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    load_env_file_locked();
    for (const auto& kv : g_table) s += kv.first + " = " + kv.second + "\n";
  }
  if (len) *len = s.size();
  if (!buf) return FK_OK;
  if (cap < s.size() + 1) return FK_EINVAL;
  std::memcpy(buf, s.c_str(), s.size() + 1);
  return FK_OK;
}

extern "C" fk_status fk_autotune_clear(void) {
  std::lock_guard<std::mutex> lk(g_tune_mu);
  g_table.clear();
  g_file_loaded = true;
  return FK_OK;
}
