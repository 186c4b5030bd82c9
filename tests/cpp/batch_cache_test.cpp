// Host-only test of the batched apply's cache policy (csrc/batch_cache.h):
// entries recorded into a caller's capture (pinned) are never evicted, only
// dropped with a plan they use.  Prints "ok" and exits 0 on success.
#include <cstdio>
#include <cstdlib>
#include <memory>
#include <set>

#include "batch_cache.h"

namespace {
std::set<int> g_alive;
int g_syncs = 0;

struct Entry {
    int id;
    bool pinned = false;
    explicit Entry(int i) : id(i) { g_alive.insert(i); }
    ~Entry() { g_alive.erase(id); }
};

#define CHECK(c)                                                         \
    do {                                                                 \
        if (!(c)) {                                                      \
            std::fprintf(stderr, "check failed line %d: %s\n", __LINE__, #c); \
            std::exit(1);                                                \
        }                                                                \
    } while (0)

bool alive(int id) { return g_alive.count(id) != 0; }
}  // namespace

int main() {
    vg::BatchCache<Entry> c;
    auto sync = [] { ++g_syncs; };
    for (int i = 0; i < 8; ++i) c.push_front(std::make_unique<Entry>(i));  // 7 is the most recent
    // entries 0 and 1 (the oldest) were recorded into a caller's capture
    c.find([](const Entry& e) { return e.id == 0; })->pinned = true;
    c.find([](const Entry& e) { return e.id == 1; })->pinned = true;
    // find moved 0 and 1 to the front; mark them old again by touching the rest
    for (int i = 2; i < 8; ++i) CHECK(c.find([i](const Entry& e) { return e.id == i; }) != nullptr);
    CHECK(c.size() == 8 && c.pinned() == 2);

    // keep 3 unpinned: the oldest unpinned (2, 3, 4) go, pinned ones stay
    CHECK(c.trim(3, sync) == 3);
    CHECK(g_syncs == 1);
    CHECK(!alive(2) && !alive(3) && !alive(4));
    CHECK(alive(0) && alive(1) && alive(5) && alive(6) && alive(7));

    // evict everything evictable: pinned entries survive any eviction
    CHECK(c.trim(0, sync) == 3);
    CHECK(alive(0) && alive(1) && c.size() == 2);
    CHECK(c.trim(0, sync) == 0);
    const int syncs = g_syncs;
    CHECK(c.evict_if([](const Entry&) { return true; }, sync) == 0);
    CHECK(g_syncs == syncs);  // nothing to free: no wait
    CHECK(alive(0) && alive(1));

    // a plan's release drops its entries, pinned or not
    c.push_front(std::make_unique<Entry>(9));
    CHECK(c.drop_if([](const Entry& e) { return e.id == 0 || e.id == 9; }, sync) == 2);
    CHECK(!alive(0) && !alive(9) && alive(1));
    CHECK(g_syncs == syncs + 1);

    // eviction with a predicate (entries on a replaced workspace) skips pinned
    c.push_front(std::make_unique<Entry>(10));
    c.push_front(std::make_unique<Entry>(11));
    CHECK(c.evict_if([](const Entry& e) { return e.id == 1 || e.id == 10; }, sync) == 1);
    CHECK(alive(1) && !alive(10) && alive(11));
    std::printf("ok\n");
    return 0;
}
