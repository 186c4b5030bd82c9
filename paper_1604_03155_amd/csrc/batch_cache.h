// Cache policy of the batched apply (host only; no HIP types, so the policy
// is also compiled and tested on its own).
//
// Entries are kept most recently used first.  An entry whose launches were
// recorded into a caller's stream capture is PINNED: the caller's graph holds
// raw pointers into the entry's device descriptors (and workspace), so
// eviction skips it; it is dropped only together with a plan it uses
// (drop_if), when the caller's graph becomes invalid anyway.
#pragma once

#include <cstddef>
#include <list>
#include <memory>

namespace vg {

template <typename Entry>
class BatchCache {
public:
    using Ptr = std::unique_ptr<Entry>;

    // The first entry satisfying pred, moved to the front; nullptr if none.
    template <typename Pred>
    Entry* find(Pred pred) {
        for (auto it = items_.begin(); it != items_.end(); ++it) {
            if (pred(**it)) {
                items_.splice(items_.begin(), items_, it);
                return items_.front().get();
            }
        }
        return nullptr;
    }

    Entry* push_front(Ptr e) {
        items_.push_front(std::move(e));
        return items_.front().get();
    }

    // Evict unpinned entries, least recently used first, until at most `keep`
    // unpinned entries remain.  before_free() runs once before the first
    // eviction (the library waits for the device there: a dropped entry's
    // graph may still be running).  Returns the number evicted.
    template <typename F>
    size_t trim(size_t keep, F&& before_free) {
        size_t unpinned = 0;
        for (const Ptr& e : items_) unpinned += e->pinned ? 0 : 1;
        size_t n = 0;
        bool synced = false;
        for (auto it = items_.end(); unpinned > keep && it != items_.begin();) {
            --it;
            if ((*it)->pinned) continue;
            if (!synced) {
                before_free();
                synced = true;
            }
            it = items_.erase(it);
            --unpinned;
            ++n;
        }
        return n;
    }

    // Evict the unpinned entries satisfying pred.
    template <typename Pred, typename F>
    size_t evict_if(Pred pred, F&& before_free) {
        return remove(before_free, [&](const Entry& e) { return !e.pinned && pred(e); });
    }

    // Drop every entry satisfying pred, pinned or not.
    template <typename Pred, typename F>
    size_t drop_if(Pred pred, F&& before_free) {
        return remove(before_free, pred);
    }

    size_t size() const { return items_.size(); }
    size_t pinned() const {
        size_t n = 0;
        for (const Ptr& e : items_) n += e->pinned ? 1 : 0;
        return n;
    }

private:
    template <typename F, typename Pred>
    size_t remove(F& before_free, Pred pred) {
        bool any = false;
        for (const Ptr& e : items_) any = any || pred(*e);
        if (!any) return 0;
        before_free();
        size_t n = 0;
        for (auto it = items_.begin(); it != items_.end();) {
            if (pred(**it)) {
                it = items_.erase(it);
                ++n;
            } else {
                ++it;
            }
        }
        return n;
    }

    std::list<Ptr> items_;
};

}  // namespace vg
