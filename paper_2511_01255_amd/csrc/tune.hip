// tune.hip -- the launch-shape cache of the tuner: a process-wide map from a
// problem key (table layout version, kind, size buckets, precision) to two
// integers, optionally persisted in the text file named by QPM_TUNE_CACHE
// ("key v0 v1" lines, appended as new shapes are measured; read when first
// needed and again whenever the variable names another file). A cached shape
// that the caller's check rejects (an old or edited file) counts as absent,
// so the caller measures again.
#include <cstdio>
#include <cstdlib>
#include <functional>
#include <map>
#include <mutex>
#include <string>

#include "common.hpp"

namespace qpm {

static std::mutex g_mu;
static std::map<std::string, std::pair<int, int>> g_map;
static std::string g_loaded_path;  // the cache file read into g_map ("" = none yet)

static int bucket(int64_t v)
{
    int b = 0;
    while ((int64_t(1) << b) < v) ++b;
    return b;
}

std::string tune_key(const char *kind, int64_t a, int64_t b, int prec, int64_t c)
{
    char buf[160];
    // the version names the kernels' table layout: shapes measured on another
    // layout are not reused
    std::snprintf(buf, sizeof(buf), "gfx950/v2/%s/a%d/b%d/p%d/c%d", kind, bucket(a), bucket(b), prec, bucket(c));
    return buf;
}

// reads the file named by QPM_TUNE_CACHE into the map when it names a file
// not read yet (its entries replace the map's for the same keys)
static void load_locked()
{
    const char *path = std::getenv("QPM_TUNE_CACHE");
    if (!path || g_loaded_path == path) return;
    g_loaded_path = path;
    FILE *fh = std::fopen(path, "r");
    if (!fh) return;
    char key[160];
    int v0, v1;
    while (std::fscanf(fh, "%159s %d %d", key, &v0, &v1) == 3) g_map[key] = {v0, v1};
    std::fclose(fh);
}

bool tune_lookup(const std::string &key, int *v0, int *v1, const std::function<bool(int, int)> &valid)
{
    std::lock_guard<std::mutex> lk(g_mu);
    load_locked();
    auto it = g_map.find(key);
    if (it == g_map.end()) return false;
    if (valid && !valid(it->second.first, it->second.second)) {
        g_map.erase(it);
        return false;
    }
    *v0 = it->second.first;
    *v1 = it->second.second;
    return true;
}

void tune_store(const std::string &key, int v0, int v1)
{
    std::lock_guard<std::mutex> lk(g_mu);
    load_locked();
    g_map[key] = {v0, v1};
    const char *path = std::getenv("QPM_TUNE_CACHE");
    if (!path) return;
    FILE *fh = std::fopen(path, "a");
    if (!fh) return;
    std::fprintf(fh, "%s %d %d\n", key.c_str(), v0, v1);
    std::fclose(fh);
}

}  // namespace qpm
