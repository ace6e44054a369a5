// tune.hpp -- process-wide table of hop launch shapes chosen by the autotuner.
#pragma once

#include "device_common.hpp"

namespace stg {

struct TuneChoice {
    int xcd_remap;
    int sites_per_thread;
    int stage_neighbours;
    int threads_per_site;
    double us;  // measured duration of one hop with this shape
};

bool tune_lookup(const Geom &g, int fmt, int nr, TuneChoice &c);
void tune_store(const Geom &g, int fmt, int nr, const TuneChoice &c);
int tune_append_file(const char *path, const Geom &g, int fmt, int nr, const TuneChoice &c);

// Fields per launch (the RHS per block): the largest number of fields one hop launch
// takes for a (lattice, link format), 1, 2, 4 or 8, chosen by the autotuner from
// the time per field of each chunking.
bool fields_lookup(const Geom &g, int fmt, int &cap);
void fields_store(const Geom &g, int fmt, int cap);
int fields_append_file(const char *path, const Geom &g, int fmt, int cap, double us_per_field);

void tune_clear();  // empties both tables
int tune_load_file(const char *path, int *loaded);

}  // namespace stg
