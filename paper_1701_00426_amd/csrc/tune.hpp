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
void tune_clear();
int tune_append_file(const char *path, const Geom &g, int fmt, int nr, const TuneChoice &c);
int tune_load_file(const char *path, int *loaded);

}  // namespace stg
