// tune.hip -- the launch-shape cache of the tuner: a process-wide map from a
// problem key (kind, size buckets, precision) to two integers, optionally
// persisted in the text file named by QPM_TUNE_CACHE ("key v0 v1" lines,
// appended as new shapes are measured).
#include <cstdio>
#include <cstdlib>
#include <map>
#include <mutex>
#include <string>

#include "common.hpp"

namespace qpm {

static std::mutex g_mu;
static std::map<std::string, std::pair<int, int>> g_map;
static bool g_loaded = false;

static int bucket(int64_t v)
{
    int b = 0;
    while ((int64_t(1) << b) < v) ++b;
    return b;
}

std::string tune_key(const char *kind, int64_t a, int64_t b, int prec, int64_t c)
{
    char buf[160];
    std::snprintf(buf, sizeof(buf), "gfx950/%s/a%d/b%d/p%d/c%d", kind, bucket(a), bucket(b), prec, bucket(c));
    return buf;
}

static void load_locked()
{
    if (g_loaded) return;
    g_loaded = true;
    const char *path = std::getenv("QPM_TUNE_CACHE");
    if (!path) return;
    FILE *fh = std::fopen(path, "r");
    if (!fh) return;
    char key[160];
    int v0, v1;
    while (std::fscanf(fh, "%159s %d %d", key, &v0, &v1) == 3) g_map[key] = {v0, v1};
    std::fclose(fh);
}

bool tune_lookup(const std::string &key, int *v0, int *v1)
{
    std::lock_guard<std::mutex> lk(g_mu);
    load_locked();
    auto it = g_map.find(key);
    if (it == g_map.end()) return false;
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
