// Launch choices that leave every result bit for bit the same (rows per
// workgroup and their order for the block mat-vec, non-temporal stores for
// the marching step), timed on the caller's own data and kept per device,
// kernel, problem size and runs per launch.  The table lives for the
// process; with KRY_TUNE_CACHE set to a file path it is read from that file
// on first use and written back after each tuning, one line per entry:
//     <device> <kernel> <n> <runs> <a> <b> <microseconds>
#include "kry_internal.h"

#include <cstdio>
#include <cstdlib>
#include <fstream>
#include <map>
#include <mutex>
#include <sstream>
#include <string>
#include <tuple>

namespace kry {

namespace {

using Key = std::tuple<std::string, std::string, int64_t, int32_t>;

struct TuneTable {
    std::mutex mu;
    bool loaded = false;
    std::map<Key, TuneChoice> entries;
};

TuneTable& table() {
    static TuneTable* t = new TuneTable();
    return *t;
}

const char* cache_path() {
    const char* p = std::getenv("KRY_TUNE_CACHE");
    return (p && *p) ? p : nullptr;
}

// caller holds the lock
void load_locked(TuneTable& t) {
    if (t.loaded) return;
    t.loaded = true;
    const char* path = cache_path();
    if (!path) return;
    std::ifstream in(path);
    std::string line;
    while (std::getline(in, line)) {
        std::istringstream ls(line);
        std::string dev, kernel;
        int64_t n = 0;
        int32_t runs = 0;
        TuneChoice c{};
        if (ls >> dev >> kernel >> n >> runs >> c.a >> c.b >> c.us) t.entries[Key{dev, kernel, n, runs}] = c;
    }
}

void save_locked(const TuneTable& t) {
    const char* path = cache_path();
    if (!path) return;
    const std::string tmp = std::string(path) + ".tmp";
    {
        std::ofstream out(tmp, std::ios::trunc);
        for (const auto& kv : t.entries) {
            const Key& k = kv.first;
            out << std::get<0>(k) << ' ' << std::get<1>(k) << ' ' << std::get<2>(k) << ' ' << std::get<3>(k) << ' '
                << kv.second.a << ' ' << kv.second.b << ' ' << kv.second.us << '\n';
        }
    }
    std::rename(tmp.c_str(), path);
}

}  // namespace

std::string tune_device_tag() {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return "unknown";
    hipDeviceProp_t prop{};
    if (hipGetDeviceProperties(&prop, dev) != hipSuccess) return "unknown";
    std::string arch(prop.gcnArchName);
    const auto colon = arch.find(':');
    if (colon != std::string::npos) arch = arch.substr(0, colon);
    return arch + "-" + std::to_string(prop.multiProcessorCount) + "cu";
}

bool tune_lookup(const std::string& kernel, int64_t n, int32_t runs, TuneChoice* out) {
    TuneTable& t = table();
    std::lock_guard<std::mutex> g(t.mu);
    load_locked(t);
    const auto it = t.entries.find(Key{tune_device_tag(), kernel, n, runs});
    if (it == t.entries.end()) return false;
    *out = it->second;
    return true;
}

void tune_store(const std::string& kernel, int64_t n, int32_t runs, const TuneChoice& c) {
    TuneTable& t = table();
    std::lock_guard<std::mutex> g(t.mu);
    load_locked(t);
    t.entries[Key{tune_device_tag(), kernel, n, runs}] = c;
    save_locked(t);
}

void tune_clear() {
    TuneTable& t = table();
    std::lock_guard<std::mutex> g(t.mu);
    t.entries.clear();
    t.loaded = false;   // the next use reads the cache file again
}

}  // namespace kry
