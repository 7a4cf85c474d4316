// Randomised check of the request loop's arena allocator against a plain
// byte-map model: no two live allocations overlap, the free list is exactly
// the complement of the live set with neighbours merged, an allocation
// succeeds whenever some free block is large enough, and allocations run
// forward from the previous one (next fit).
#include <cstdio>
#include <cstdlib>
#include <random>
#include <vector>

#include "arena.h"

#define CHECK(c)                                                               \
    do {                                                                       \
        if (!(c)) {                                                            \
            std::fprintf(stderr, "check failed at line %d: %s\n", __LINE__, #c); \
            return 1;                                                          \
        }                                                                      \
    } while (0)

int main() {
    const uint64_t size = 1 << 16;
    for (int seed = 0; seed < 60; seed++) {
        std::mt19937_64 rng(seed);
        aesgpu::Arena arena(size);
        std::vector<int> owner(size, -1);
        struct Live { uint64_t off, n; };
        std::vector<Live> live;
        uint64_t last_end = 0;
        for (int step = 0; step < 2000; step++) {
            if (live.empty() || rng() % 3) {
                const uint64_t n = 1 + rng() % 3000;
                bool any = false;
                for (auto &b : arena.free_blocks())
                    any |= b.second >= n;
                // next fit: when the space right after the previous
                // allocation is free, the new one must start there
                bool room_at_cursor = last_end + n <= size;
                for (uint64_t i = last_end; room_at_cursor && i < last_end + n; i++)
                    room_at_cursor = owner[i] < 0;
                uint64_t off = 0;
                const bool ok = arena.alloc(n, &off);
                CHECK(ok == any);
                if (!ok)
                    continue;
                CHECK(off + n <= size);
                for (uint64_t i = off; i < off + n; i++) {
                    CHECK(owner[i] < 0);
                    owner[i] = step;
                }
                if (room_at_cursor)
                    CHECK(off == last_end);
                last_end = off + n;
                live.push_back({off, n});
            } else {
                const size_t k = rng() % live.size();
                for (uint64_t i = live[k].off; i < live[k].off + live[k].n; i++)
                    owner[i] = -1;
                arena.release(live[k].off, live[k].n);
                live.erase(live.begin() + k);
            }
            // the free list is exactly the complement, with neighbours merged
            uint64_t pos = 0, prev_end = ~uint64_t(0);
            for (auto &b : arena.free_blocks()) {
                CHECK(b.second > 0);
                CHECK(b.first != prev_end);
                for (uint64_t i = pos; i < b.first; i++)
                    CHECK(owner[i] >= 0);
                for (uint64_t i = b.first; i < b.first + b.second; i++)
                    CHECK(owner[i] < 0);
                pos = prev_end = b.first + b.second;
            }
            for (uint64_t i = pos; i < size; i++)
                CHECK(owner[i] >= 0);
        }
    }
    std::printf("arena ok\n");
    return 0;
}
