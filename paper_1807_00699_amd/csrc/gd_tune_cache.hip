// Persistent cache of the variant tuners (dense coupling kernels and batched
// solver).  With GD_AUTOTUNE_CACHE=<file> the variant a tuner picked for a
// problem key is stored in the file, and the tuners look a key up there first
// (re-reading the file whenever its size or modification time changed, so
// other processes' picks are seen) before their in-process table or timing.  The file's first line names the device
// (architecture, compute units) and this library build (its variant counts
// and build stamp); a file with another first line is ignored and rewritten
// on the next store.  Each further line: "<kind> <key fields...> <variant id>".
// The callers check every id they read against the problem (fits) and tune
// again when it does not fit.  Stores replace the file atomically (a
// temporary file renamed over it); two processes storing at once may each
// drop the other's new entry, which then is tuned again.  Host code only.
#include "gd_internal.h"

#include <sys/stat.h>
#include <unistd.h>

#include <cstdio>
#include <cstdlib>
#include <fstream>
#include <map>
#include <mutex>
#include <sstream>
#include <string>
#include <vector>

namespace gd {

namespace {

std::mutex g_mu;
std::string g_path;
long long g_size = -1, g_mtime = -1;       // of the file when last read or written
std::map<std::string, int> g_entries;

std::string header() {
    int dev = 0;
    hipDeviceProp_t p{};
    std::string arch = "unknown";
    int cus = 0;
    if (hipGetDevice(&dev) == hipSuccess && hipGetDeviceProperties(&p, dev) == hipSuccess) {
        arch = p.gcnArchName;
        for (char &c : arch)
            if (c == ' ') c = '_';
        cus = p.multiProcessorCount;
    }
    std::ostringstream h;
    h << "gd-autotune 1 " << arch << " " << cus << " variants " << dense_config_count(false) << ","
      << dense_config_count(true) << "," << dense_lp_config_count() << "," << gemv_config_count() << ","
      << batch_config_count() << " build " << __DATE__ << "_" << __TIME__;
    return h.str();
}

std::string entry_key(const char *kind, const std::vector<long long> &key) {
    std::ostringstream o;
    o << kind;
    for (long long v : key) o << " " << v;
    return o.str();
}

bool file_stamp(const std::string &path, long long &size, long long &mtime) {
    struct stat st;
    if (stat(path.c_str(), &st) != 0) return false;
    size = (long long)st.st_size;
    mtime = (long long)st.st_mtim.tv_sec * 1000000000LL + st.st_mtim.tv_nsec;
    return true;
}

// (under g_mu) the file named by GD_AUTOTUNE_CACHE, read again when it changed
void load_locked() {
    const char *p = std::getenv("GD_AUTOTUNE_CACHE");
    if (!p || !*p) {
        g_path.clear();
        g_entries.clear();
        return;
    }
    long long size = -1, mtime = -1;
    const bool exists = file_stamp(p, size, mtime);
    if (g_path == p && size == g_size && mtime == g_mtime) return;
    g_path = p;
    g_size = size;
    g_mtime = mtime;
    g_entries.clear();
    if (!exists) return;
    std::ifstream in(g_path);
    std::string line;
    if (!in || !std::getline(in, line) || line != header()) return;
    while (std::getline(in, line)) {
        const size_t sp = line.find_last_of(' ');
        if (sp == std::string::npos) continue;
        char *end = nullptr;
        const long id = std::strtol(line.c_str() + sp + 1, &end, 10);
        if (end == line.c_str() + sp + 1 || *end != '\0') continue;
        g_entries[line.substr(0, sp)] = int(id);
    }
}

}  // namespace

int tune_cache_lookup(const char *kind, const std::vector<long long> &key) {
    std::lock_guard<std::mutex> lk(g_mu);
    load_locked();
    auto it = g_entries.find(entry_key(kind, key));
    return it == g_entries.end() ? -1 : it->second;
}

void tune_cache_store(const char *kind, const std::vector<long long> &key, int id) {
    std::lock_guard<std::mutex> lk(g_mu);
    load_locked();
    if (g_path.empty()) return;
    const std::string k = entry_key(kind, key);
    g_entries[k] = id;
    // write the whole file (the header of this device and build, then every
    // entry) under a temporary name and rename it over the old one, so that
    // another process reading the file sees either version whole
    const std::string tmp = g_path + ".tmp" + std::to_string((long long)getpid());
    bool ok;
    {
        std::ofstream out(tmp, std::ios::trunc);
        if (!out) return;
        out << header() << "\n";
        for (const auto &e : g_entries) out << e.first << " " << e.second << "\n";
        out.flush();
        ok = bool(out);
    }
    if (!ok || std::rename(tmp.c_str(), g_path.c_str()) != 0) {
        std::remove(tmp.c_str());
        return;
    }
    file_stamp(g_path, g_size, g_mtime);
}

}  // namespace gd
