// tune_cache.hip -- the autotuners' choice cache, in memory and optionally in
// a file (see tune_cache.hpp).
#include "tune_cache.hpp"

#include <cstdio>
#include <cstdlib>
#include <map>
#include <mutex>
#include <sstream>

namespace stn {

namespace {

std::mutex g_mu;
std::map<std::string, std::vector<int>> g_map;
bool g_loaded = false;

const char *cache_path()
{
    const char *p = std::getenv("STENCIL_TUNE_CACHE");
    return p && *p ? p : nullptr;
}

// caller holds g_mu
void load_once()
{
    if (g_loaded)
        return;
    g_loaded = true;
    const char *path = cache_path();
    if (!path)
        return;
    FILE *f = std::fopen(path, "r");
    if (!f)
        return;
    char line[1024];
    while (std::fgets(line, sizeof(line), f)) {
        std::istringstream in(line);
        std::string key;
        if (!(in >> key))
            continue;
        std::vector<int> vals;
        int v;
        while (in >> v)
            vals.push_back(v);
        if (!vals.empty())
            g_map[key] = vals;
    }
    std::fclose(f);
}

} // namespace

bool tune_cache_get(const std::string &key, std::vector<int> &vals)
{
    std::lock_guard<std::mutex> lk(g_mu);
    load_once();
    auto it = g_map.find(key);
    if (it == g_map.end())
        return false;
    vals = it->second;
    return true;
}

void tune_cache_put(const std::string &key, const std::vector<int> &vals)
{
    std::lock_guard<std::mutex> lk(g_mu);
    load_once();
    g_map[key] = vals;
    const char *path = cache_path();
    if (!path)
        return;
    FILE *f = std::fopen(path, "a");
    if (!f)
        return;
    std::fprintf(f, "%s", key.c_str());
    for (int v : vals)
        std::fprintf(f, " %d", v);
    std::fprintf(f, "\n");
    std::fclose(f);
}

} // namespace stn
