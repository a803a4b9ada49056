// Admission policy of the served path, free of device calls so that it runs
// (and is tested) on the host alone. The serving loop supplies the device
// work; this header decides where a submitted W goes and which queued
// requests join the running batch.
//
// Rules:
//   - a request's device region (W plus its instance state) comes from a
//     first-fit range allocator over the context arena;
//   - regions are handed out in submission order: a new request takes one at
//     submission only when no earlier request is waiting for one, and
//     admission stops at the first queued request whose region does not fit
//     (no later request overtakes it);
//   - a W that cannot be staged in the pinned ring and finds no free region
//     is refused (back-pressure) unless there is no ring at all;
//   - at most max_batch requests are in the batch (running or loading).
#pragma once
#include <cstddef>
#include <deque>
#include <vector>

#include "sk_alloc.h"

namespace sk {

// Where a submitted request's W goes.
enum class Entry {
    Again,          // refused for now: queue full, or neither ring room nor a region
    RingAndDevice,  // staged in the pinned ring, copied to its region at once
    RingOnly,       // staged in the ring, waits in the queue for a region
    DeviceOnly,     // no ring room: copied straight into a free region
    Heap            // no ring at all and no free region: staged on the heap
};

struct EntryPlan {
    Entry kind = Entry::Again;
    size_t ring_off = 0, dev_off = 0;  // valid for the kinds that use them
};

// ring: the pinned ring's allocator, or nullptr when there is no ring.
// queued: requests waiting in the queue; staged_waiting: those of them
// whose W is still in host staging (without a region). wbytes: staged size
// of W; len: device footprint. Whatever the plan uses is allocated here;
// nothing is allocated for Entry::Again.
inline EntryPlan plan_entry(RangeAlloc *ring, RangeAlloc &dev, size_t queued, size_t max_queue,
                            int staged_waiting, size_t wbytes, size_t len) {
    EntryPlan e;
    if (queued >= max_queue) return e;
    const bool in_ring = ring != nullptr && ring->alloc(wbytes, e.ring_off);
    const bool placed = staged_waiting == 0 && dev.alloc(len, e.dev_off);
    if (in_ring) e.kind = placed ? Entry::RingAndDevice : Entry::RingOnly;
    else if (placed) e.kind = Entry::DeviceOnly;
    else e.kind = ring != nullptr ? Entry::Again : Entry::Heap;
    return e;
}

// Moves queued requests into the batch in FIFO order while it has room
// (in_flight = requests running or loading). R has `bool copying` (its W is
// on its way to its region), `bool loaded` (its W is in its region),
// `size_t len` and `int phase`. A request without a region gets one here
// (place(r, offset) carves it; staged_waiting drops by one) and goes to
// to_copy; one whose copy is in flight goes to to_copy as well; one already
// loaded goes to fresh. Stops at the first request whose region does not fit.
template <class R, class Place>
inline void admit_fifo(std::deque<R *> &queue, size_t in_flight, size_t max_batch, RangeAlloc &dev,
                       int &staged_waiting, std::vector<R *> &fresh, std::vector<R *> &to_copy,
                       Place place) {
    while (!queue.empty() && in_flight + fresh.size() + to_copy.size() < max_batch) {
        R *r = queue.front();
        if (r->copying) {
            to_copy.push_back(r);
        } else if (!r->loaded) {
            size_t off;
            if (!dev.alloc(r->len, off)) break;
            place(r, off);
            --staged_waiting;
            to_copy.push_back(r);
        } else {
            fresh.push_back(r);
        }
        r->phase = 1;
        queue.pop_front();
    }
}

}  // namespace sk
