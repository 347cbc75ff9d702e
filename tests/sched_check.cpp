// Unit checks of the serving loop's scheduling policy (paper_1206_3316_amd/csrc/
// dmc_sched.cpp), built with the address and undefined-behaviour sanitizers by
// tests/test_host_sched.py.  Prints "ok" and exits 0 when every check holds.
#include <cstdio>
#include <algorithm>
#include <cstdlib>
#include <random>
#include <vector>

#include "dmc_sched.h"

using namespace dmc::sched;

static int failures = 0;
#define CHECK(c)                                                         \
    do {                                                                 \
        if (!(c)) {                                                      \
            std::fprintf(stderr, "%s:%d: check failed: %s\n", __FILE__, __LINE__, #c); \
            ++failures;                                                  \
        }                                                                \
    } while (0)

static void arena_random_sequences()
{
    std::mt19937_64 rng(12345);
    for (int trial = 0; trial < 200; ++trial) {
        const size_t size = 256 * (1 + rng() % 4096);
        Arena a(size);
        CHECK(a.consistent() && a.free_bytes() == size);
        std::vector<std::pair<size_t, size_t>> live;  // (off, bytes)
        for (int step = 0; step < 400; ++step) {
            if (live.empty() || rng() % 3) {
                const size_t want = 1 + rng() % (size / 4 + 1);
                size_t off = 0;
                if (a.alloc(want, off)) {
                    const size_t g = (want + 255) & ~size_t(255);
                    CHECK(off % 256 == 0 && off + g <= size);
                    for (auto &l : live) CHECK(off + g <= l.first || l.first + l.second <= off);  // no overlap
                    live.emplace_back(off, g);
                } else {
                    CHECK(a.largest_free() < ((want + 255) & ~size_t(255)));  // first fit fails only if nothing fits
                }
            } else {
                const size_t k = rng() % live.size();
                CHECK(a.release(live[k].first));
                CHECK(!a.release(live[k].first));  // a second release of the same range is refused
                live.erase(live.begin() + (long)k);
            }
            CHECK(a.consistent());
            size_t used = 0;
            for (auto &l : live) used += l.second;
            CHECK(a.free_bytes() + used == size);
            CHECK(a.live_ranges() == live.size());
        }
        for (auto &l : live) CHECK(a.release(l.first));
        CHECK(a.consistent() && a.free_bytes() == size && a.largest_free() == size);  // fully coalesced
    }
    Arena z(100);  // smaller than one granule: nothing fits
    size_t off = 0;
    CHECK(!z.alloc(1, off) && z.consistent());
    CHECK(!z.release(0));
}

static void admission_in_arrival_order()
{
    Arena a(256 * 10);
    size_t want[5] = {256 * 4, 256 * 4, 256 * 4, 256, 256};
    size_t off[5];
    // the third request does not fit: admission stops there (the small ones behind it wait)
    CHECK(admit(a, want, 5, 0, 8, off) == 2);
    CHECK(off[0] == 0 && off[1] == 256 * 4);
    // slots: at most max_active - n_active
    Arena b(256 * 100);
    CHECK(admit(b, want, 5, 6, 8, off) == 2);
    CHECK(admit(b, want, 5, 8, 8, off) == 0);
    CHECK(admit(b, want, 0, 0, 8, off) == 0);
    // after a release the waiting head fits (first fit: the freed range), then the rest behind it
    CHECK(a.release(0));
    CHECK(admit(a, want + 2, 3, 2, 8, off) == 3 && off[0] == 0 && off[1] == 256 * 8 && off[2] == 256 * 9);
    CHECK(a.consistent() && a.free_bytes() == 0);
}

static void group_round_robin()
{
    bool has[4] = {false, true, false, true};
    CHECK(next_group(has, 4, 0) == 1);
    CHECK(next_group(has, 4, 2) == 3);
    CHECK(next_group(has, 4, 4) == 1);  // wraps
    bool none[4] = {false, false, false, false};
    CHECK(next_group(none, 4, 1) == -1);
    bool one[1] = {true};
    CHECK(next_group(one, 1, 0) == 0);
}

static void slices()
{
    CHECK(slice(2e10, 4, 100.0, 1ull << 40) == 50000000ull);
    CHECK(slice(2e10, 4, 1e12, 1ull << 40) == 256);   // at least 256 particles
    CHECK(slice(2e10, 4, 100.0, 1000) == 1000);        // at most what is left
    CHECK(slice(2e10, 0, 100.0, 1000) == 1000);        // no members: no division by zero
    CHECK(slice(1e30, 1, 1e-300, 7) == 7);             // no overflow of the conversion
    CHECK(slice(2e10, 3, 5.0, 0) == 0);
}

// Shortest-remaining-first slices: the epoch's budget is what equal shares would
// run, and it goes to the members with the fewest flights left first.
static void shortest_first_slices()
{
    {
        // remaining flights 1e9, 3e10, 5e9, 0 (suspended particles only); share 5e9
        const double fpp[4] = {100.0, 100.0, 50.0, 100.0};
        const uint64_t left[4] = {10000000ull, 300000000ull, 100000000ull, 0ull};
        uint64_t out[4];
        slices(2e10, 4, fpp, left, out);
        // budget = 1e9 + 5e9 + 5e9 + 0 = 1.1e10: member 3 (nothing left) takes none,
        // member 0 all of its 1e9, member 2 all of its 5e9, member 1 the 5e9 left
        CHECK(out[3] == 0 && out[0] == 10000000ull && out[2] == 100000000ull && out[1] == 50000000ull);
        double run = 0.0, eq = 0.0;
        for (int i = 0; i < 4; ++i) {
            run += out[i] * fpp[i];
            eq += (double)slice(2e10, 4, fpp[i], left[i]) * fpp[i];
            CHECK(out[i] <= left[i]);
        }
        CHECK(run == 1.1e10 && eq == 1.1e10);  // as long as the equal-share epoch
    }
    {
        // every member larger than its share: the smallest takes the whole budget
        const double fpp[3] = {10.0, 10.0, 10.0};
        const uint64_t left[3] = {9000000000ull, 3000000000ull, 6000000000ull};
        uint64_t out[3];
        slices(3e9, 3, fpp, left, out);
        CHECK(out[1] == 300000000ull && out[0] == 0 && out[2] == 0);
    }
    {
        // ties keep member order; the 256-particle floor holds while budget lasts
        const double fpp[3] = {1e9, 1e9, 1e9};
        const uint64_t left[3] = {1000, 1000, 1000};
        uint64_t out[3];
        slices(3e9, 3, fpp, left, out);  // share 1e9 = one particle each, budget 3e9
        CHECK(out[0] == 256 && out[1] == 0 && out[2] == 0);
    }
    {
        uint64_t out[1] = {7};
        slices(2e10, 0, nullptr, nullptr, out);  // no members: nothing touched
        CHECK(out[0] == 7);
    }
    // random members: never more than left, never negative budget overrun beyond
    // one member's 256-particle floor, and the members served form a prefix of the
    // order by remaining flights
    std::mt19937_64 rng(777);
    for (int trial = 0; trial < 500; ++trial) {
        const size_t n = 1 + rng() % 32;
        std::vector<double> fpp(n);
        std::vector<uint64_t> left(n), out(n);
        for (size_t i = 0; i < n; ++i) {
            fpp[i] = 1.0 + (double)(rng() % 5000);
            left[i] = (rng() % 4 == 0) ? 0 : rng() % 100000000ull;
        }
        const double E = 1e6 * (double)(1 + rng() % 100000);
        slices(E, n, fpp.data(), left.data(), out.data());
        double budget = 0.0, run = 0.0, fmax = 0.0;
        for (size_t i = 0; i < n; ++i) {
            budget += std::min((double)left[i] * fpp[i], E / (double)n);
            run += (double)out[i] * fpp[i];
            fmax = std::max(fmax, fpp[i]);
            CHECK(out[i] <= left[i]);
        }
        CHECK(run <= budget + 256.0 * fmax);
        for (size_t i = 0; i < n; ++i)
            for (size_t j = 0; j < n; ++j) {
                // a member with fewer flights left is served in full before one with more starts
                const double wi = (double)left[i] * fpp[i], wj = (double)left[j] * fpp[j];
                if (wi < wj && out[j] > 0) CHECK(out[i] == left[i]);
            }
    }
}

static void resume_mapping()
{
    int r0, r1, r2, r3;
    const void *prev[3] = {&r0, &r1, &r2};
    uint64_t susp[3] = {5, 0, 2};
    const void *now[3] = {&r3, &r2, &r0};
    int32_t map[8];
    CHECK(resume_map(prev, susp, 3, now, 3, map, 8));
    CHECK(map[0] == 2 && map[1] == 0 && map[2] == 1 && map[3] == 0);
    // r1 left nothing suspended: it may be gone (collected) without harm
    const void *now2[2] = {&r0, &r2};
    CHECK(resume_map(prev, susp, 3, now2, 2, map, 8));
    // r2 left particles suspended but is not a member now: refused
    const void *now3[2] = {&r0, &r3};
    CHECK(!resume_map(prev, susp, 3, now3, 2, map, 8));
    CHECK(!resume_map(prev, susp, 3, now, 3, map, 2));  // table too short
    CHECK(resume_map(prev, susp, 0, now, 0, map, 8));   // first epoch of a group
}

int main()
{
    arena_random_sequences();
    admission_in_arrival_order();
    group_round_robin();
    slices();
    shortest_first_slices();
    resume_mapping();
    if (failures) {
        std::fprintf(stderr, "%d checks failed\n", failures);
        return 1;
    }
    std::printf("ok\n");
    return 0;
}
