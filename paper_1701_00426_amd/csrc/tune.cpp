// tune.cpp -- launch-shape autotuner of the hop kernels.
//
// The paper fixes its OpenACC tile sizes per architecture at compile time, after
// measuring which sizes run fastest on each machine (Sec. 4.3, TILE0..2; Sec. 5).
// Here the launch shape of the hop is chosen at run time: for a (lattice, link
// format, fields-per-launch) key the autotuner times every candidate shape on the
// caller's buffers with HIP events, keeps the fastest in a process-wide table that
// every hop launch consults, and appends it to a cache file (one JSON object per
// line) that a later process can load.  A second table holds, per (lattice, link
// format), how many fields one launch takes at most (the RHS per block): the
// chunking of several fields into launches with the least time per field.  Results
// never depend on either choice.

#include <hip/hip_runtime.h>

#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <tuple>

#include "tune.hpp"

namespace stg {

namespace {

using Key = std::tuple<uint32_t, uint32_t, uint32_t, uint32_t, int, int>;

std::mutex g_mu;
std::map<Key, TuneChoice> g_table;
std::map<Key, int> g_fields;  // key with nr = 0

Key make_key(const Geom &g, int fmt, int nr) {
    return Key(g.N[0], g.N[1], g.N[2], g.N[3], fmt, nr);
}

}  // namespace

bool tune_lookup(const Geom &g, int fmt, int nr, TuneChoice &c) {
    std::lock_guard<std::mutex> lk(g_mu);
    auto it = g_table.find(make_key(g, fmt, nr));
    if (it == g_table.end()) return false;
    c = it->second;
    return true;
}

void tune_store(const Geom &g, int fmt, int nr, const TuneChoice &c) {
    std::lock_guard<std::mutex> lk(g_mu);
    g_table[make_key(g, fmt, nr)] = c;
}

bool fields_lookup(const Geom &g, int fmt, int &cap) {
    std::lock_guard<std::mutex> lk(g_mu);
    auto it = g_fields.find(make_key(g, fmt, 0));
    if (it == g_fields.end()) return false;
    cap = it->second;
    return true;
}

void fields_store(const Geom &g, int fmt, int cap) {
    std::lock_guard<std::mutex> lk(g_mu);
    g_fields[make_key(g, fmt, 0)] = cap;
}

void tune_clear() {
    std::lock_guard<std::mutex> lk(g_mu);
    g_table.clear();
    g_fields.clear();
}

int fields_append_file(const char *path, const Geom &g, int fmt, int cap, double us_per_field) {
    FILE *f = std::fopen(path, "a");
    if (!f) return -1;
    std::fprintf(f,
                 "{\"arch\": \"gfx950\", \"dims\": [%u, %u, %u, %u], \"fmt\": %d, "
                 "\"fields_per_launch\": %d, \"us_per_field\": %.3f}\n",
                 g.N[0], g.N[1], g.N[2], g.N[3], fmt, cap, us_per_field);
    std::fclose(f);
    return 0;
}

int tune_append_file(const char *path, const Geom &g, int fmt, int nr, const TuneChoice &c) {
    FILE *f = std::fopen(path, "a");
    if (!f) return -1;
    std::fprintf(f,
                 "{\"arch\": \"gfx950\", \"dims\": [%u, %u, %u, %u], \"fmt\": %d, \"nr\": %d, "
                 "\"xcd_remap\": %d, \"sites_per_thread\": %d, \"stage_neighbours\": %d, "
                 "\"threads_per_site\": %d, \"us\": %.3f}\n",
                 g.N[0], g.N[1], g.N[2], g.N[3], fmt, nr, c.xcd_remap, c.sites_per_thread,
                 c.stage_neighbours, c.threads_per_site, c.us);
    std::fclose(f);
    return 0;
}

namespace {

// Value of "key": <number> in one cache line; false when the key is absent.
bool find_num(const char *line, const char *key, double &v) {
    char pat[64];
    std::snprintf(pat, sizeof pat, "\"%s\": ", key);
    const char *p = std::strstr(line, pat);
    if (!p) return false;
    char *end = nullptr;
    v = std::strtod(p + std::strlen(pat), &end);
    return end != p + std::strlen(pat);
}

bool find_int(const char *line, const char *key, int &v) {
    double d;
    if (!find_num(line, key, d) || d != (double)(int)d) return false;
    v = (int)d;
    return true;
}

}  // namespace

int tune_load_file(const char *path, int *loaded) {
    FILE *f = std::fopen(path, "r");
    if (!f) return -1;
    char line[512];
    int n = 0;
    while (std::fgets(line, sizeof line, f)) {
        unsigned d[4];
        int fmt, nr, xcd, spt, stage = 0, tps = 1;
        double us;
        if (!std::strstr(line, "\"arch\": \"gfx950\"")) continue;
        const char *dims = std::strstr(line, "\"dims\": [");
        if (!dims || std::sscanf(dims, "\"dims\": [%u, %u, %u, %u]", &d[0], &d[1], &d[2], &d[3]) != 4)
            continue;
        Geom g;
        std::memset(&g, 0, sizeof g);
        for (int k = 0; k < 4; ++k) g.N[k] = d[k];
        if (std::strstr(line, "\"fields_per_launch\"")) {
            int cap;
            if (!find_int(line, "fmt", fmt) || !find_int(line, "fields_per_launch", cap) ||
                (cap != 1 && cap != 2 && cap != 4 && cap != 8))
                continue;
            fields_store(g, fmt, cap);  // later lines win
            ++n;
            continue;
        }
        if (!find_int(line, "fmt", fmt) || !find_int(line, "nr", nr) ||
            !find_int(line, "xcd_remap", xcd) || !find_int(line, "sites_per_thread", spt) ||
            !find_num(line, "us", us))
            continue;
        // fields added later are optional: lines without them read as their defaults
        if (std::strstr(line, "\"stage_neighbours\"") && !find_int(line, "stage_neighbours", stage))
            continue;
        if (std::strstr(line, "\"threads_per_site\"") && !find_int(line, "threads_per_site", tps))
            continue;
        if ((xcd != 0 && xcd != 1) || (spt != 1 && spt != 2 && spt != 4 && spt != 8) ||
            (stage != 0 && stage != 1) || (tps != 1 && tps != 2 && tps != 4))
            continue;
        tune_store(g, fmt, nr, TuneChoice{xcd, spt, stage, tps, us});  // later lines win
        ++n;
    }
    std::fclose(f);
    if (loaded) *loaded = n;
    return 0;
}

}  // namespace stg
