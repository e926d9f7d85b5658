// Persistent table of measured launch shapes: 1D level-step tilings (per n, boundary and PCR
// stage count), the grouped 1D tiling, and the 2D transform-pass shapes (per n and precision).
//
// The autotuners record their choices here; the table is loaded on first use from a JSON file
// and the file is rewritten after every new entry, so later processes reuse the measurements.
// File: $RIDC_TUNE_CACHE if set ("" or "off": no file), else $XDG_CACHE_HOME/ridc/tune.json,
// else $HOME/.cache/ridc/tune.json.  The file names the GPU it was measured on (architecture
// and compute-unit count); entries of another GPU are not loaded.
#include <sys/stat.h>
#include <unistd.h>

#include <cerrno>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <string>

#include "ridc_internal.h"

namespace ridc {

namespace {

struct Rec1D {
  int64_t n;
  int bc, stages, threads, rows, flags;
};
struct Rec2D {
  int64_t n;
  int prec, tile;
};

struct Store {
  std::mutex mu;
  bool loaded = false;
  std::vector<Rec1D> t1;
  bool has_batch = false;
  int batch_threads = 0, batch_rows = 0;
  std::vector<Rec2D> t2;
};

Store& store() {
  static Store s;
  return s;
}

std::string device_id() {
  int dev = 0;
  hipDeviceProp_t prop;
  if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&prop, dev) != hipSuccess) {
    (void)hipGetLastError();
    return "";
  }
  std::string arch = prop.gcnArchName;
  const size_t colon = arch.find(':');
  if (colon != std::string::npos) arch.resize(colon);
  return arch + "/" + std::to_string(prop.multiProcessorCount);
}

std::string default_path() {
  const char* env = std::getenv("RIDC_TUNE_CACHE");
  if (env) return (!*env || std::strcmp(env, "off") == 0) ? "" : env;
  const char* xdg = std::getenv("XDG_CACHE_HOME");
  if (xdg && *xdg) return std::string(xdg) + "/ridc/tune.json";
  const char* home = std::getenv("HOME");
  if (home && *home) return std::string(home) + "/.cache/ridc/tune.json";
  return "";
}

void make_parent_dirs(const std::string& path) {
  for (size_t i = 1; i < path.size(); ++i)
    if (path[i] == '/') {
      const std::string d = path.substr(0, i);
      if (mkdir(d.c_str(), 0755) != 0 && errno != EEXIST) return;
    }
}

// the flat objects {"k": integer, ...} of the array named `key`
std::vector<std::map<std::string, int64_t>> objects(const std::string& s, const char* key) {
  std::vector<std::map<std::string, int64_t>> out;
  const std::string k = std::string("\"") + key + "\"";
  size_t p = s.find(k);
  if (p == std::string::npos) return out;
  p = s.find_first_of("[{", p + k.size());
  if (p == std::string::npos) return out;
  const bool array = s[p] == '[';
  const size_t end = array ? s.find(']', p) : s.find('}', p) + 1;
  if (end == std::string::npos) return out;
  size_t q = p;
  while (true) {
    const size_t a = s.find('{', q);
    if (a == std::string::npos || a >= end) break;
    const size_t b = s.find('}', a);
    if (b == std::string::npos || b > end) break;
    std::map<std::string, int64_t> obj;
    size_t r = a;
    while (true) {
      const size_t k0 = s.find('"', r);
      if (k0 == std::string::npos || k0 > b) break;
      const size_t k1 = s.find('"', k0 + 1);
      if (k1 == std::string::npos || k1 > b) break;
      const size_t c = s.find(':', k1);
      if (c == std::string::npos || c > b) break;
      char* stop = nullptr;
      const long long v = std::strtoll(s.c_str() + c + 1, &stop, 10);
      if (stop == s.c_str() + c + 1) break;
      obj[s.substr(k0 + 1, k1 - k0 - 1)] = v;
      r = (size_t)(stop - s.c_str());
    }
    out.push_back(obj);
    q = b + 1;
    if (!array) break;
  }
  return out;
}

std::string string_field(const std::string& s, const char* key) {
  const std::string k = std::string("\"") + key + "\"";
  size_t p = s.find(k);
  if (p == std::string::npos) return "";
  p = s.find('"', s.find(':', p + k.size()));
  if (p == std::string::npos) return "";
  const size_t e = s.find('"', p + 1);
  return e == std::string::npos ? "" : s.substr(p + 1, e - p - 1);
}

// Merge the entries of `path` into the table (caller holds the lock).  Returns false when the
// file cannot be read; a file of another GPU adds nothing.
bool load_locked(Store& st, const std::string& path) {
  FILE* f = std::fopen(path.c_str(), "rb");
  if (!f) return false;
  std::string s;
  char buf[4096];
  size_t got;
  while ((got = std::fread(buf, 1, sizeof buf, f)) > 0) s.append(buf, got);
  std::fclose(f);
  const std::string dev = device_id();
  if (!dev.empty() && string_field(s, "device") != dev) return true;
  auto has = [](const std::map<std::string, int64_t>& o, std::initializer_list<const char*> ks) {
    for (const char* k : ks)
      if (!o.count(k)) return false;
    return true;
  };
  for (auto& o : objects(s, "tile1d")) {
    if (!has(o, {"n", "bc", "stages", "threads", "rows", "flags"})) continue;
    Rec1D r{o["n"], (int)o["bc"], (int)o["stages"], (int)o["threads"], (int)o["rows"],
            (int)o["flags"]};
    bool found = false;
    for (auto& e : st.t1)
      if (e.n == r.n && e.bc == r.bc && e.stages == r.stages) {
        e = r;
        found = true;
      }
    if (!found) st.t1.push_back(r);
  }
  for (auto& o : objects(s, "batch1d"))
    if (has(o, {"threads", "rows"})) {
      st.has_batch = true;
      st.batch_threads = (int)o["threads"];
      st.batch_rows = (int)o["rows"];
    }
  for (auto& o : objects(s, "pass2d")) {
    if (!has(o, {"n", "prec", "tile"})) continue;
    Rec2D r{o["n"], (int)o["prec"], (int)o["tile"]};
    bool found = false;
    for (auto& e : st.t2)
      if (e.n == r.n && e.prec == r.prec) {
        e = r;
        found = true;
      }
    if (!found) st.t2.push_back(r);
  }
  return true;
}

bool save_locked(const Store& st, const std::string& path) {
  make_parent_dirs(path);
  const std::string tmp = path + ".tmp" + std::to_string((long long)getpid());
  FILE* f = std::fopen(tmp.c_str(), "wb");
  if (!f) return false;
  std::fprintf(f, "{\n  \"format\": \"ridc-tune-1\",\n  \"device\": \"%s\",\n",
               device_id().c_str());
  std::fprintf(f, "  \"tile1d\": [");
  for (size_t i = 0; i < st.t1.size(); ++i) {
    const Rec1D& r = st.t1[i];
    std::fprintf(f, "%s\n    {\"n\": %lld, \"bc\": %d, \"stages\": %d, \"threads\": %d, "
                 "\"rows\": %d, \"flags\": %d}", i ? "," : "", (long long)r.n, r.bc, r.stages,
                 r.threads, r.rows, r.flags);
  }
  std::fprintf(f, "\n  ],\n");
  if (st.has_batch)
    std::fprintf(f, "  \"batch1d\": {\"threads\": %d, \"rows\": %d},\n", st.batch_threads,
                 st.batch_rows);
  std::fprintf(f, "  \"pass2d\": [");
  for (size_t i = 0; i < st.t2.size(); ++i)
    std::fprintf(f, "%s\n    {\"n\": %lld, \"prec\": %d, \"tile\": %d}", i ? "," : "",
                 (long long)st.t2[i].n, st.t2[i].prec, st.t2[i].tile);
  std::fprintf(f, "\n  ]\n}\n");
  const bool ok = std::fclose(f) == 0;
  if (!ok || std::rename(tmp.c_str(), path.c_str()) != 0) {
    std::remove(tmp.c_str());
    return false;
  }
  return true;
}

// First use: load the default file.
Store& ready() {
  Store& st = store();
  if (!st.loaded) {
    st.loaded = true;
    const std::string p = default_path();
    if (!p.empty()) (void)load_locked(st, p);
  }
  return st;
}

void persist_locked(const Store& st) {
  const std::string p = default_path();
  if (!p.empty()) (void)save_locked(st, p);   // a cache that cannot be written is not an error
}

}  // namespace

bool tune_get_1d(int64_t n, int bc, int stages, int* threads, int* rows, int* flags) {
  std::lock_guard<std::mutex> lk(store().mu);
  Store& st = ready();
  for (auto& e : st.t1)
    if (e.n == n && e.bc == bc && e.stages == stages) {
      *threads = e.threads;
      *rows = e.rows;
      *flags = e.flags;
      return true;
    }
  return false;
}

void tune_put_1d(int64_t n, int bc, int stages, int threads, int rows, int flags) {
  std::lock_guard<std::mutex> lk(store().mu);
  Store& st = ready();
  bool found = false;
  for (auto& e : st.t1)
    if (e.n == n && e.bc == bc && e.stages == stages) {
      e = Rec1D{n, bc, stages, threads, rows, flags};
      found = true;
    }
  if (!found) st.t1.push_back(Rec1D{n, bc, stages, threads, rows, flags});
  persist_locked(st);
}

bool tune_get_batch(int* threads, int* rows) {
  std::lock_guard<std::mutex> lk(store().mu);
  Store& st = ready();
  if (!st.has_batch) return false;
  *threads = st.batch_threads;
  *rows = st.batch_rows;
  return true;
}

void tune_put_batch(int threads, int rows) {
  std::lock_guard<std::mutex> lk(store().mu);
  Store& st = ready();
  st.has_batch = true;
  st.batch_threads = threads;
  st.batch_rows = rows;
  persist_locked(st);
}

bool tune_get_2d(int64_t n, int prec, int* tile) {
  std::lock_guard<std::mutex> lk(store().mu);
  Store& st = ready();
  for (auto& e : st.t2)
    if (e.n == n && e.prec == prec) {
      *tile = e.tile;
      return true;
    }
  return false;
}

void tune_put_2d(int64_t n, int prec, int tile) {
  std::lock_guard<std::mutex> lk(store().mu);
  Store& st = ready();
  bool found = false;
  for (auto& e : st.t2)
    if (e.n == n && e.prec == prec) {
      e.tile = tile;
      found = true;
    }
  if (!found) st.t2.push_back(Rec2D{n, prec, tile});
  persist_locked(st);
}

int tune_save(const char* path) {
  std::lock_guard<std::mutex> lk(store().mu);
  Store& st = ready();
  const std::string p = path ? path : default_path();
  if (p.empty()) return fail(RIDC_E_INVAL, "no tuning cache file (RIDC_TUNE_CACHE is off)");
  if (!save_locked(st, p)) return fail(RIDC_E_INVAL, "cannot write " + p);
  return RIDC_OK;
}

int tune_load(const char* path) {
  std::lock_guard<std::mutex> lk(store().mu);
  Store& st = ready();
  const std::string p = path ? path : default_path();
  if (p.empty()) return fail(RIDC_E_INVAL, "no tuning cache file (RIDC_TUNE_CACHE is off)");
  if (!load_locked(st, p)) return fail(RIDC_E_INVAL, "cannot read " + p);
  return RIDC_OK;
}

void tune_clear() {
  std::lock_guard<std::mutex> lk(store().mu);
  Store& st = store();
  st.loaded = true;            // do not reload the file after a clear
  st.t1.clear();
  st.t2.clear();
  st.has_batch = false;
}

}  // namespace ridc
