// dmc_sched.cpp -- the serving loop's scheduling policy (see dmc_sched.h).
#include "dmc_sched.h"

#include <algorithm>
#include <iterator>
#include <vector>

namespace dmc {
namespace sched {

namespace {
size_t granule(size_t x) { return (x + 255) & ~size_t(255); }
}  // namespace

Arena::Arena(size_t size) : size_(size & ~size_t(255))
{
    if (size_) free_[0] = size_;
}

bool Arena::alloc(size_t bytes, size_t &off)
{
    if (bytes == 0) bytes = 1;
    if (bytes > size_) return false;
    bytes = granule(bytes);
    for (auto it = free_.begin(); it != free_.end(); ++it) {
        if (it->second >= bytes) {
            off = it->first;
            const size_t rest = it->second - bytes;
            free_.erase(it);
            if (rest) free_[off + bytes] = rest;
            used_[off] = bytes;
            return true;
        }
    }
    return false;
}

bool Arena::release(size_t off)
{
    auto u = used_.find(off);
    if (u == used_.end()) return false;
    size_t start = off, len = u->second;
    used_.erase(u);
    auto next = free_.lower_bound(start);
    if (next != free_.end() && start + len == next->first) {
        len += next->second;
        next = free_.erase(next);
    }
    if (next != free_.begin()) {
        auto prev = std::prev(next);
        if (prev->first + prev->second == start) {
            start = prev->first;
            len += prev->second;
            free_.erase(prev);
        }
    }
    free_[start] = len;
    return true;
}

size_t Arena::free_bytes() const
{
    size_t s = 0;
    for (const auto &f : free_) s += f.second;
    return s;
}

size_t Arena::largest_free() const
{
    size_t m = 0;
    for (const auto &f : free_) m = std::max(m, f.second);
    return m;
}

bool Arena::consistent() const
{
    // merge both maps in address order: ranges must tile [0, size) exactly
    std::map<size_t, std::pair<size_t, bool>> all;  // start -> (length, free)
    for (const auto &f : free_) {
        if (f.second == 0 || !all.emplace(f.first, std::make_pair(f.second, true)).second) return false;
    }
    for (const auto &u : used_) {
        if (u.second == 0 || !all.emplace(u.first, std::make_pair(u.second, false)).second) return false;
    }
    size_t at = 0;
    bool prev_free = false;
    for (const auto &r : all) {
        if (r.first != at) return false;
        if (r.second.second && prev_free) return false;  // two free neighbours: not coalesced
        if (r.first % 256 != 0 || r.second.first % 256 != 0) return false;
        at = r.first + r.second.first;
        prev_free = r.second.second;
    }
    return at == size_;
}

int admit(Arena &arena, const size_t *pending_bytes, int n_pending, int n_active, int max_active, size_t *off)
{
    int n = 0;
    while (n < n_pending && n_active + n < max_active) {
        if (!arena.alloc(pending_bytes[n], off[n])) break;
        ++n;
    }
    return n;
}

int next_group(const bool *has, int n_classes, int next_class)
{
    for (int k = 0; k < n_classes; ++k) {
        const int c = ((next_class % n_classes) + n_classes + k) % n_classes;
        if (has[c]) return c;
    }
    return -1;
}

uint64_t slice(double epoch_flights, size_t n_members, double flights_per_particle, uint64_t left)
{
    const double share = epoch_flights / (double)std::max<size_t>(n_members, 1);
    const double want = std::max(256.0, share / std::max(flights_per_particle, 1e-300));
    const uint64_t n = want >= 1.8e19 ? UINT64_MAX : (uint64_t)want;
    return std::min(n, left);
}

void slices(double epoch_flights, size_t n, const double *flights_per_particle, const uint64_t *left,
            uint64_t *out)
{
    const double share = epoch_flights / (double)std::max<size_t>(n, 1);
    std::vector<double> work(n);
    std::vector<size_t> order(n);
    double budget = 0.0;
    for (size_t i = 0; i < n; ++i) {
        work[i] = (double)left[i] * std::max(flights_per_particle[i], 0.0);
        budget += std::min(work[i], share);
        order[i] = i;
    }
    std::stable_sort(order.begin(), order.end(), [&](size_t a, size_t b) { return work[a] < work[b]; });
    for (size_t i : order) {
        out[i] = budget > 0.0 ? slice(budget, 1, flights_per_particle[i], left[i]) : 0;
        // a member that cannot take all it has left used up the budget
        budget = out[i] < left[i] ? 0.0 : budget - (double)out[i] * flights_per_particle[i];
    }
}

bool resume_map(const void *const *prev_members, const uint64_t *prev_suspended, size_t n_prev,
                const void *const *members, size_t n_members, int32_t *resume_job, size_t resume_len)
{
    if (n_prev > resume_len) return false;
    for (size_t i = 0; i < resume_len; ++i) resume_job[i] = 0;
    for (size_t i = 0; i < n_prev; ++i) {
        if (prev_suspended[i] == 0) continue;  // no particle carries this slot
        int32_t idx = -1;
        for (size_t j = 0; j < n_members; ++j)
            if (members[j] == prev_members[i]) idx = (int32_t)j;
        if (idx < 0) return false;
        resume_job[i] = idx;
    }
    return true;
}

}  // namespace sched
}  // namespace dmc
