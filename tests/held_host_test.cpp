// Host-only check of the out-of-core brick store: random hold / merge / release sequences against
// a std::map model (every held entry's 512 words intact, blocks never shared, released blocks
// reused before new chunks), then clear().  Built with g++ and the address/undefined-behaviour
// sanitizers by test_held_host.py.
#include <cstdio>
#include <cstring>
#include <map>
#include <random>
#include <set>
#include <vector>

#include "../paper_2605_26325_amd/csrc/dare_held.h"

#define CHECK(c)                                                    \
    do {                                                            \
        if (!(c)) {                                                 \
            std::fprintf(stderr, "check failed line %d: %s\n", __LINE__, #c); \
            return 1;                                               \
        }                                                           \
    } while (0)

int main() {
    using Block = std::vector<unsigned long long>;
    constexpr size_t W = dare::HeldStore::kBlockWords;
    dare::HeldStore st;
    std::map<int64_t, Block> model;
    std::mt19937_64 rng(11);
    size_t peak = 0;
    for (int step = 0; step < 60000; ++step) {
        const int op = (int)(rng() % 100);
        const int64_t e = (int64_t)(rng() % 9000);
        if (op < 55) {   // hold: a fresh block, or add into the held one
            Block acc(W);
            for (auto& x : acc) x = rng() & 0xFFFFFFFFull;
            bool fresh = false;
            unsigned long long* b = st.add(e, fresh);
            CHECK(b != nullptr);
            CHECK(fresh == (model.count(e) == 0));
            if (fresh) {
                std::memcpy(b, acc.data(), W * sizeof(unsigned long long));
                model[e] = acc;
            } else {
                Block& m = model[e];
                for (size_t k = 0; k < W; ++k) {
                    b[k] += acc[k];
                    m[k] += acc[k];
                }
            }
        } else if (op < 85) {   // release
            st.erase(e);
            model.erase(e);
            CHECK(st.find(e) == nullptr);
        } else {   // look up
            unsigned long long* b = st.find(e);
            CHECK((b != nullptr) == (model.count(e) != 0));
            if (b) CHECK(std::memcmp(b, model[e].data(), W * sizeof(unsigned long long)) == 0);
        }
        CHECK(st.size() == model.size());
        peak = model.size() > peak ? model.size() : peak;
        if (step % 5000 == 0) {   // every held entry intact, no two sharing a block
            std::set<const unsigned long long*> seen;
            for (auto& kv : model) {
                unsigned long long* b = st.find(kv.first);
                CHECK(b != nullptr && seen.insert(b).second);
                CHECK(std::memcmp(b, kv.second.data(), W * sizeof(unsigned long long)) == 0);
            }
            CHECK(st.index().size() == model.size());
        }
    }
    CHECK(peak > dare::HeldStore::kChunkBlocks);   // more than one chunk was in use
    st.clear();
    CHECK(st.empty() && st.find(1) == nullptr);
    bool fresh = false;
    CHECK(st.add(5, fresh) != nullptr && fresh && st.size() == 1);
    std::printf("held host test ok (peak %zu entries)\n", peak);
    return 0;
}
