// Host-only test of the persistent autotuner cache (csrc/tune_cache.cpp):
// round trip, and a missing, corrupt or stale file (or out-of-range values)
// read as "no entry", so the plan tunes or keeps its defaults.
// Usage: tune_cache_test <scratch directory>.  Prints "ok" on success.
#include <cstdio>
#include <cstdlib>
#include <fstream>
#include <string>

#include "tune_cache.h"

#define CHECK(c)                                                              \
    do {                                                                      \
        if (!(c)) {                                                           \
            std::fprintf(stderr, "check failed line %d: %s\n", __LINE__, #c); \
            std::exit(1);                                                     \
        }                                                                     \
    } while (0)

static void write(const std::string& path, const std::string& text) {
    std::ofstream o(path, std::ios::binary | std::ios::trunc);
    o << text;
}

int main(int argc, char** argv) {
    CHECK(argc == 2);
    const std::string dir = argv[1];
    const std::string path = dir + "/sub/dir/tune.json";  // parent directories are created
    const std::string key = "d=3;N=256;table=complex;precision=fp32;mode=quick;device=gfx950/256cu;build=abc";
    const std::string other = "d=3;N=256;table=complex;precision=fp32;mode=quick;device=gfx950/256cu;build=OLD";
    vg::TuneChoice c;

    // missing file
    CHECK(!vg::tune_cache_lookup(path, key, &c));
    // disabled cache (empty path)
    CHECK(!vg::tune_cache_lookup("", key, &c));
    CHECK(!vg::tune_cache_store("", key, c));

    // round trip
    vg::TuneChoice a;
    a.pad_bytes = 512;
    a.xcd_map = 0;
    a.fs_L1 = 256;
    a.generic = 0;
    a.ms = 0.7123;
    CHECK(vg::tune_cache_store(path, key, a));
    vg::TuneChoice b;
    CHECK(vg::tune_cache_lookup(path, key, &b));
    CHECK(b.pad_bytes == 512 && b.xcd_map == 0 && b.fs_L1 == 256 && b.generic == 0 && b.ms == 0.7123);

    // a second key leaves the first in place; stale (other build) keys are not matched
    vg::TuneChoice d;
    d.pad_bytes = 0;
    CHECK(vg::tune_cache_store(path, other, d));
    CHECK(vg::tune_cache_lookup(path, key, &b) && b.pad_bytes == 512);
    CHECK(vg::tune_cache_lookup(path, other, &b) && b.pad_bytes == 0);
    CHECK(!vg::tune_cache_lookup(path, key + "x", &b));

    // corrupt files of several kinds: no entry
    const char* corrupt[] = {
        "",
        "{",
        "not json",
        "{\"format\": \"vgconv-tune-1\", \"entries\": {\"" ,
        "{\"format\": \"other-format\", \"entries\": {}}",
        "{\"format\": \"vgconv-tune-1\"}",
        "{\"format\": \"vgconv-tune-1\", \"entries\": []}",
        "[1, 2, 3]",
        "{\"format\": \"vgconv-tune-1\", \"entries\": {}} trailing",
    };
    for (const char* t : corrupt) {
        write(path, t);
        CHECK(!vg::tune_cache_lookup(path, key, &b));
    }
    // truncated copy of a valid file
    CHECK(vg::tune_cache_store(path, key, a));
    {
        std::ifstream in(path);
        std::string text((std::istreambuf_iterator<char>(in)), std::istreambuf_iterator<char>());
        write(path, text.substr(0, text.size() / 2));
    }
    CHECK(!vg::tune_cache_lookup(path, key, &b));
    // a store over a corrupt file replaces it with a valid one
    CHECK(vg::tune_cache_store(path, key, a));
    CHECK(vg::tune_cache_lookup(path, key, &b) && b.pad_bytes == 512);

    // values outside the search space, or missing fields: no entry
    const char* bad[] = {
        "\"pad_bytes\": 300, \"xcd_map\": 1, \"fs_L1\": 0, \"generic\": 0",
        "\"pad_bytes\": 256, \"xcd_map\": 2, \"fs_L1\": 0, \"generic\": 0",
        "\"pad_bytes\": 256, \"xcd_map\": 1, \"fs_L1\": 7, \"generic\": 0",
        "\"pad_bytes\": 256, \"xcd_map\": 1, \"fs_L1\": 0, \"generic\": -1",
        "\"pad_bytes\": 256.5, \"xcd_map\": 1, \"fs_L1\": 0, \"generic\": 0",
        "\"xcd_map\": 1, \"fs_L1\": 0, \"generic\": 0",
        "\"pad_bytes\": \"256\", \"xcd_map\": 1, \"fs_L1\": 0, \"generic\": 0",
    };
    for (const char* f : bad) {
        write(path, std::string("{\"format\": \"vgconv-tune-1\", \"entries\": {\"") + key + "\": {" + f + "}}}");
        CHECK(!vg::tune_cache_lookup(path, key, &b));
    }
    // unknown extra fields are ignored
    write(path, std::string("{\"format\": \"vgconv-tune-1\", \"note\": [true, null], \"entries\": {\"") + key +
                    "\": {\"pad_bytes\": 1024, \"xcd_map\": 1, \"fs_L1\": 32, \"generic\": 1, \"x\": \"y\"}}}");
    CHECK(vg::tune_cache_lookup(path, key, &b));
    CHECK(b.pad_bytes == 1024 && b.fs_L1 == 32 && b.generic == 1 && b.ms == 0.0);
    std::printf("ok\n");
    return 0;
}
