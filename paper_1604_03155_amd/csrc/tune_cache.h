// Persistent cache of the autotuner's choices (host only; no HIP types, so it
// is also compiled and tested on its own).
//
// A JSON file maps a key naming everything the choice depends on -- grid
// (d, N), table class, precision, tune mode, device (architecture and
// compute-unit count) and the library build -- to the chosen layout:
//
//   {"format": "vgconv-tune-1",
//    "entries": {"<key>": {"pad_bytes": 256, "xcd_map": 1, "fs_L1": 0,
//                          "generic": 0, "ms": 0.7123}, ...}}
//
// A missing, unreadable or corrupt file, a key that is absent (another device
// or library build: stale), or an entry whose values are outside the tuner's
// search space are all treated as "no entry", and the plan tunes (or keeps
// its defaults).  Stores rewrite the whole file through a temporary file and
// a rename, so a reader never sees a half-written file; a corrupt file is
// replaced by one holding only the new entry.
#pragma once

#include <string>

namespace vg {

struct TuneChoice {
    int pad_bytes = 256;
    int xcd_map = 1;
    int fs_L1 = 0;
    int generic = 0;
    double ms = 0.0;  // measured time per apply (informational)
};

// Cache file path: $VG_TUNE_CACHE if set (empty: caching disabled, returns
// ""), else $XDG_CACHE_HOME/vgconv/tune.json, else $HOME/.cache/vgconv/tune.json.
std::string tune_cache_path();

// Whether `c` lies in the tuner's search space.
bool tune_choice_valid(const TuneChoice& c);

// Look up `key` in the file at `path`; false if there is no usable entry.
bool tune_cache_lookup(const std::string& path, const std::string& key, TuneChoice* out);

// Add or replace `key`; false if the file could not be written (the caller
// ignores it: the plan is tuned either way).
bool tune_cache_store(const std::string& path, const std::string& key, const TuneChoice& c);

}  // namespace vg
