// Host-only check of the serving arena's first-fit allocator: random
// allocate/release sequences against a byte-ownership map (no overlap, exact
// accounting, full coalescing once everything is released).  Built with g++
// and the address/undefined-behaviour sanitizers by test_alloc_host.py.
#include <cstdio>
#include <cstdlib>
#include <random>
#include <vector>

#include "../paper_2605_26325_amd/csrc/dare_alloc.h"

#define CHECK(c)                                                    \
    do {                                                            \
        if (!(c)) {                                                 \
            std::fprintf(stderr, "check failed line %d: %s\n", __LINE__, #c); \
            return 1;                                               \
        }                                                           \
    } while (0)

int main() {
    const uint64_t base = 4096, size = 1 << 20, align = 256;
    dare::RangeAlloc a(base, size, align);
    CHECK(a.capacity() == size);
    std::vector<int> owner(size / align, -1);
    struct Blk { uint64_t off, bytes; };
    std::vector<Blk> live;
    std::mt19937_64 rng(7);
    int next = 0;
    for (int step = 0; step < 200000; ++step) {
        const bool do_alloc = live.empty() || (rng() % 100) < 55;
        if (do_alloc) {
            const uint64_t bytes = 1 + rng() % (64 * 1024);
            const uint64_t off = a.alloc(bytes);
            if (off == UINT64_MAX) continue;   // full or fragmented: fine, just not over-committed
            CHECK(off >= base && off + bytes <= base + size && off % align == 0);
            const uint64_t u0 = (off - base) / align, u1 = (off - base + bytes + align - 1) / align;
            for (uint64_t u = u0; u < u1; ++u) {
                CHECK(owner[u] == -1);
                owner[u] = next;
            }
            live.push_back({off, bytes});
            ++next;
        } else {
            const size_t k = rng() % live.size();
            const Blk b = live[k];
            live[k] = live.back();
            live.pop_back();
            const uint64_t u0 = (b.off - base) / align, u1 = (b.off - base + b.bytes + align - 1) / align;
            for (uint64_t u = u0; u < u1; ++u) owner[u] = -1;
            a.release(b.off, b.bytes);
        }
        uint64_t used = 0;
        if (step % 997 == 0) {
            for (int o : owner) used += (o != -1) * align;
            CHECK(used == a.used());
        }
    }
    for (const Blk& b : live) a.release(b.off, b.bytes);
    CHECK(a.used() == 0);
    CHECK(a.free_ranges() == 1);
    CHECK(a.alloc(size) == base);          // the whole range coalesced back
    CHECK(a.alloc(1) == UINT64_MAX);
    CHECK(!a.fits_ever(size + 1));
    std::printf("alloc host test ok (%d allocations)\n", next);
    return 0;
}
