// dmc_sched.h -- host-side scheduling policy of the serving loop, as pure
// functions of plain values (no device, no HIP headers), so that the policy can
// be unit-tested on the CPU under the address and undefined-behaviour
// sanitizers.
//
// The serving loop (dmc_server.cpp) keeps requests in a FIFO; it admits them in
// arrival order while a slot is free and their device tallies fit a first-fit
// arena carved out of one allocation; each epoch takes the admitted requests of
// one group (every request in group 0, or one class at a time, the classes in
// turn), runs as many estimated flights as equal shares would, handed out to the
// members nearest completion first, and maps the particles its group suspended in
// its previous epoch back onto the new epoch's job table.
#pragma once

#include <cstddef>
#include <cstdint>
#include <map>

namespace dmc {
namespace sched {

// First-fit allocator over [0, size) in 256-byte granules; freed ranges
// coalesce with their free neighbours.
class Arena {
public:
    explicit Arena(size_t size);
    // Offset of a range of at least `bytes` (rounded up to 256), or false.
    bool alloc(size_t bytes, size_t &off);
    // Returns the range that starts at off; false if off is not a live range.
    bool release(size_t off);
    size_t size() const { return size_; }
    size_t free_bytes() const;
    size_t largest_free() const;
    size_t live_ranges() const { return used_.size(); }
    // Every free and used range lies in [0, size), none overlaps another, no two
    // free ranges touch (coalescing), and together they cover [0, size).
    bool consistent() const;

private:
    size_t size_;
    std::map<size_t, size_t> free_, used_;
};

// Admission in arrival order: requests [0, n_pending) of the FIFO with the
// given byte sizes are admitted while fewer than max_active are active and the
// arena has room; the first request that does not fit stops admission (no
// overtaking, so a large request is not starved).  off[i] receives the arena
// offsets of the admitted ones.  Returns how many were admitted.
int admit(Arena &arena, const size_t *pending_bytes, int n_pending, int n_active, int max_active, size_t *off);

// The group of the next epoch: the first class at or after next_class (round
// robin over n_classes) that has an admitted request; -1 if none has.
int next_group(const bool *has, int n_classes, int next_class);

// Particles a member starts in an epoch: an equal share of the epoch's
// estimated flights over the members, divided by its flights per particle; at
// least 256 and at most the particles it has left.
uint64_t slice(double epoch_flights, size_t n_members, double flights_per_particle, uint64_t left);

// Particles each of n members starts in an epoch (out[i]).  The epoch runs the
// estimated flights that equal shares would, the sum over members of
// min(remaining flights, epoch_flights / n) (remaining = left x flights per
// particle), so it is as long as with equal shares; they go to the members in
// order of remaining flights, smallest first (ties in member order), each taking
// slice(budget left, 1, ...) until one cannot take all it has left, which spends
// the budget; later members start none this epoch.  Requests nearest completion finish first, which shortens the
// latency of most requests when sizes are heavy-tailed.
void slices(double epoch_flights, size_t n, const double *flights_per_particle, const uint64_t *left,
            uint64_t *out);

// Resumed particles carry the slot (member index) of the epoch that suspended
// them.  resume_job[i] receives the index in this epoch's members of previous
// member i, for every previous member that left particles suspended (others
// get 0: no particle carries their slot).  Returns false if a previous member
// with suspended particles is not a member now (its particles would be lost).
// Previous members are identified by opaque keys and never dereferenced: a
// member whose particles all finished may have been collected since.
bool resume_map(const void *const *prev_members, const uint64_t *prev_suspended, size_t n_prev,
                const void *const *members, size_t n_members, int32_t *resume_job, size_t resume_len);

}  // namespace sched
}  // namespace dmc
