// Host-only test of the serving loop's request store and scratch budget:
// many batches submitted, admitted, delivered and released keep the store
// bounded; results survive until released; failed reservations defer a
// query without dropping it.  Exits non-zero with a message on failure.
#include <cstdio>
#include <cstdlib>
#include <vector>

#include "serve_store.h"

using namespace seismic;

#define CHECK(c)                                                              \
    do {                                                                      \
        if (!(c)) {                                                           \
            std::fprintf(stderr, "%s:%d: check failed: %s\n", __FILE__, __LINE__, #c); \
            std::exit(1);                                                     \
        }                                                                     \
    } while (0)

static ServeRequest make(uint32_t nnz, double nb) {
    ServeRequest r;
    r.words.assign(nnz, 7u);
    r.not_before = nb;
    return r;
}

int main() {
    const uint32_t k = 10;
    // 1. a long run: 200k queries in waves of 1000, at most 4 batches of 64
    //    in flight; the caller releases every delivered wave
    {
        RequestStore st;
        uint64_t max_held = 0, max_words = 0;
        std::vector<uint32_t> ids(k, 1);
        std::vector<float> sc(k, 1.0f);
        for (int wave = 0; wave < 200; ++wave) {
            for (int i = 0; i < 1000; ++i) st.submit(make(50 + i % 150, wave));
            while (st.has_pending()) {
                std::vector<uint64_t> batch;
                while (st.has_pending() && batch.size() < 64) batch.push_back(st.admit());
                uint64_t words = 0;
                for (uint64_t t = st.base(); t < st.end(); ++t) words += st.get(t)->words.size();
                if (words > max_words) max_words = words;
                for (uint64_t t : batch) st.deliver(t, ids.data(), sc.data(), k, 1.0);
                if (st.held() > max_held) max_held = st.held();
            }
            const uint64_t end = st.end();
            CHECK(st.release(end) == end);
            CHECK(st.held() == 0);
        }
        CHECK(st.completed() == 200000);
        CHECK(st.end() == 200000);
        CHECK(max_held <= 1000);
        // words of admitted requests are gone: only the wave's queued ones remain
        CHECK(max_words <= 1000ull * 200);
    }
    // 2. release stops at the first ticket that is not done
    {
        RequestStore st;
        for (int i = 0; i < 10; ++i) st.submit(make(5, 0.0));
        std::vector<uint32_t> ids(k, 3);
        std::vector<float> sc(k, 2.0f);
        for (int i = 0; i < 10; ++i) st.admit();
        for (uint64_t t : {0, 1, 2, 4}) st.deliver(t, ids.data(), sc.data(), k, 1.0);
        CHECK(st.release(10) == 3);
        CHECK(st.get(2) == nullptr && st.get(3) != nullptr && st.get(4)->done);
        CHECK(st.get(4)->ids[0] == 3 && st.get(4)->scores[9] == 2.0f);
        CHECK(st.get(3)->words.empty());  // admitted: words dropped
        CHECK(st.held() == 7);
        // submissions keep counting tickets after a release
        CHECK(st.submit(make(3, 0.0)) == 10);
        CHECK(st.last_not_before() == 0.0);
    }
    // 3. scratch budget: injected failures and a real budget defer queries,
    //    and every query is admitted in order once scratch frees up
    {
        const uint64_t one = query_scratch_bytes(100, k, 10, 400);
        CHECK(one == 400 + 160 + 32000);
        ScratchBudget b(3 * one, 2);
        CHECK(!b.reserve(one) && !b.reserve(one));  // the two injected failures
        CHECK(b.reserve(one) && b.reserve(one) && b.reserve(one));
        CHECK(!b.reserve(1));                      // budget held
        CHECK(b.failed() == 3 && b.peak() == 3 * one);
        b.release(one);
        CHECK(b.reserve(one));
        ScratchBudget unlimited(0, 0);
        for (int i = 0; i < 1000; ++i) CHECK(unlimited.reserve(one));

        RequestStore st;
        ScratchBudget bb(2 * one, 3);
        for (int i = 0; i < 20; ++i) st.submit(make(100, 0.0));
        std::vector<uint64_t> order;
        std::vector<uint64_t> inflight;
        std::vector<uint32_t> ids(k, 0);
        std::vector<float> sc(k, 0.0f);
        int attempts = 0;
        while (st.completed() < 20) {
            ++attempts;
            CHECK(attempts < 1000);
            // admission attempt: reserve one query at a time, stop at the first failure
            while (st.has_pending()) {
                if (!bb.reserve(query_scratch_bytes((uint32_t)st.pending().words.size(), k, 10, 400))) break;
                uint64_t t = st.admit();
                order.push_back(t);
                inflight.push_back(t);
            }
            // complete the oldest in-flight query
            if (!inflight.empty()) {
                st.deliver(inflight.front(), ids.data(), sc.data(), k, 0.0);
                inflight.erase(inflight.begin());
                bb.release(one);
            }
        }
        CHECK(order.size() == 20);
        for (size_t i = 0; i < order.size(); ++i) CHECK(order[i] == i);  // deferred, never dropped or reordered
        CHECK(bb.failed() >= 3);
        CHECK(bb.peak() <= 2 * one);
    }
    std::printf("serve store ok\n");
    return 0;
}
