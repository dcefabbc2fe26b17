// Autotuned launch shapes: a JSON cache keyed by (device architecture,
// image size and bands, connectivity, mode), read once per process and
// written by gapd_autotune (capi.cpp), which times the candidates.
//
// File format (one object per key):
//   {"gfx950/128x128x1/c4/m1": {"fill_lanes": 128, "walk_pf": 16, "spec_cap": 32,
//                               "naive_pfw": 4, "naive_check1": 1, "ms": 1103.2}, ...}
#include <dlfcn.h>

#include <cctype>
#include <cstdio>
#include <cstdlib>
#include <fstream>
#include <map>
#include <mutex>
#include <sstream>
#include <string>

#include "capi_internal.h"
#include "gapd_internal.h"

namespace gapd {

namespace {

struct Entry {
    Tuning t;
    double ms = 0;
};

std::mutex g_mu;
std::map<std::string, Entry> g_cache;
bool g_loaded = false;

std::string cache_path() {
    const char *env = std::getenv("GAPD_TUNE_FILE");
    if (env && *env) return env;
    Dl_info info{};
    if (dladdr((void *)&cache_path, &info) && info.dli_fname) {
        std::string so = info.dli_fname;
        const size_t slash = so.rfind('/');
        return (slash == std::string::npos ? std::string(".") : so.substr(0, slash)) + "/gapd_tune.json";
    }
    return "gapd_tune.json";
}

// The value of "name": <integer or number> inside one entry's text.
bool field(const std::string &obj, const char *name, double *v) {
    const std::string q = std::string("\"") + name + "\"";
    const size_t at = obj.find(q);
    if (at == std::string::npos) return false;
    size_t p = obj.find(':', at + q.size());
    if (p == std::string::npos) return false;
    char *end = nullptr;
    const double x = std::strtod(obj.c_str() + p + 1, &end);
    if (end == obj.c_str() + p + 1) return false;
    *v = x;
    return true;
}

void load_locked() {
    g_loaded = true;
    std::ifstream f(cache_path());
    if (!f) return;
    std::stringstream ss;
    ss << f.rdbuf();
    const std::string s = ss.str();
    size_t p = 0;
    for (;;) {
        // "key": { ... }
        const size_t k0 = s.find('"', p);
        if (k0 == std::string::npos) break;
        const size_t k1 = s.find('"', k0 + 1);
        if (k1 == std::string::npos) break;
        const size_t o0 = s.find('{', k1);
        const size_t o1 = o0 == std::string::npos ? o0 : s.find('}', o0);
        if (o1 == std::string::npos) break;
        const std::string key = s.substr(k0 + 1, k1 - k0 - 1), obj = s.substr(o0, o1 - o0 + 1);
        Entry e;
        double v;
        if (field(obj, "fill_lanes", &v)) e.t.fill_lanes = (int)v;
        if (field(obj, "walk_pf", &v)) e.t.walk_pf = (int)v;
        if (field(obj, "spec_cap", &v)) e.t.spec_cap = (int)v;
        if (field(obj, "naive_pfw", &v)) e.t.naive_pfw = (int)v;
        if (field(obj, "naive_check1", &v)) e.t.naive_check1 = (int)v;
        if (field(obj, "ms", &v)) e.ms = v;
        // Shapes the kernels do not have fall back to the defaults.
        const Tuning d;
        if (e.t.fill_lanes != 128 && e.t.fill_lanes != 256) e.t.fill_lanes = d.fill_lanes;
        if (e.t.walk_pf != 8 && e.t.walk_pf != 16) e.t.walk_pf = d.walk_pf;
        if (e.t.spec_cap < 1 || e.t.spec_cap > kSpecK) e.t.spec_cap = d.spec_cap;
        if (e.t.naive_pfw != 4 && e.t.naive_pfw != 8) e.t.naive_pfw = d.naive_pfw;
        if (e.t.naive_check1 != 0 && e.t.naive_check1 != 1) e.t.naive_check1 = d.naive_check1;
        if (key.find('/') != std::string::npos) g_cache[key] = e;
        p = o1 + 1;
    }
}

void save_locked() {
    const std::string path = cache_path(), tmp = path + ".tmp";
    std::ofstream f(tmp);
    if (!f) return;
    f << "{\n";
    size_t i = 0;
    for (const auto &kv : g_cache) {
        const Tuning &t = kv.second.t;
        char line[512];
        std::snprintf(line, sizeof line,
                      "  \"%s\": {\"fill_lanes\": %d, \"walk_pf\": %d, \"spec_cap\": %d, \"naive_pfw\": %d, "
                      "\"naive_check1\": %d, \"ms\": %.3f}%s\n",
                      kv.first.c_str(), t.fill_lanes, t.walk_pf, t.spec_cap, t.naive_pfw, t.naive_check1, kv.second.ms,
                      ++i < g_cache.size() ? "," : "");
        f << line;
    }
    f << "}\n";
    f.close();
    std::rename(tmp.c_str(), path.c_str());
}

// The current device's architecture name (gcnArchName up to its first ':'),
// looked up once per device.
std::string arch_name() {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return "unknown";
    static std::mutex mu;
    static std::map<int, std::string> names;
    std::lock_guard<std::mutex> lk(mu);
    const auto it = names.find(dev);
    if (it != names.end()) return it->second;
    hipDeviceProp_t prop{};
    if (hipGetDeviceProperties(&prop, dev) != hipSuccess) return "unknown";
    std::string a = prop.gcnArchName;
    const size_t colon = a.find(':');
    if (colon != std::string::npos) a = a.substr(0, colon);
    names[dev] = a;
    return a;
}

}  // namespace

std::string tune_key(int H, int W, int C, int conn, int mode) {
    char buf[160];
    std::snprintf(buf, sizeof buf, "%s/%dx%dx%d/c%d/m%d", arch_name().c_str(), H, W, C, conn, mode);
    return buf;
}

Tuning tuning_for(const std::string &key) {
    std::lock_guard<std::mutex> lk(g_mu);
    if (!g_loaded) load_locked();
    const auto it = g_cache.find(key);
    return it == g_cache.end() ? Tuning() : it->second.t;
}

void store_tuning(const std::string &key, const Tuning &t, double ms, bool save) {
    std::lock_guard<std::mutex> lk(g_mu);
    if (!g_loaded) load_locked();
    g_cache[key] = Entry{t, ms};
    if (save) save_locked();
}

}  // namespace gapd
