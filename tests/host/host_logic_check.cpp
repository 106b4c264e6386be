// Host-only checks of paper_1711_05152_amd/csrc/host_logic.h, built with a host compiler under
// AddressSanitizer and UndefinedBehaviorSanitizer by tests/test_host_sanitized.py (no GPU, no HIP).
// Prints "ok <check>" per passed check and the random-stream values the test compares with the
// oracle's independent implementation; exits non-zero on the first failed check.
#include <stdio.h>
#include <stdlib.h>

#include <random>
#include <set>
#include <vector>

#include "host_logic.h"

using namespace mr1l::host;

#define CHECK(cond)                                                              \
    do {                                                                         \
        if (!(cond)) {                                                           \
            fprintf(stderr, "check failed at line %d: %s\n", __LINE__, #cond);   \
            exit(1);                                                             \
        }                                                                        \
    } while (0)

static void check_rows() {
    std::mt19937_64 g(7);
    for (int rep = 0; rep < 300; ++rep) {
        const int d = 1 + (int)(g() % 6);
        const int64_t n = (int64_t)(g() % 200);
        std::vector<int32_t> f((size_t)n * d);
        for (auto& v : f) v = (int32_t)(g() % 5) - 2;   // small box: duplicates are common
        // brute force: the first pair (in input order of the later row) of equal rows
        bool dup = false;
        for (int64_t i = 0; i < n && !dup; ++i)
            for (int64_t j = i + 1; j < n && !dup; ++j) {
                bool eq = true;
                for (int c = 0; c < d; ++c) eq = eq && f[i * d + c] == f[j * d + c];
                dup = eq;
            }
        int64_t a = -1, b = -1;
        const bool got = find_equal_rows(f.data(), n, d, &a, &b);
        CHECK(got == dup);
        if (got) {
            CHECK(0 <= a && a < b && b < n);
            for (int c = 0; c < d; ++c) CHECK(f[a * d + c] == f[b * d + c]);
        }
    }
    printf("ok distinct_rows\n");
}

static void check_primes() {
    const int N = 200000;
    std::vector<char> comp(N + 1, 0);
    for (int i = 2; (int64_t)i * i <= N; ++i)
        if (!comp[i])
            for (int j = i * i; j <= N; j += i) comp[j] = 1;
    for (int p = -3; p <= N; ++p) CHECK(is_prime(p) == (p >= 2 && !comp[p]));
    // prime sizes above lambda, with an injectivity predicate that rejects every third prime
    std::vector<int64_t> got;
    int k = 0;
    CHECK(prime_sizes(1000.5, 12, [&](int64_t) { return (k++ % 3 == 2) ? 0 : 1; }, got) == 0);
    std::vector<int64_t> want;
    k = 0;
    for (int p = 1001; (int)want.size() < 12; ++p)
        if (p >= 2 && !comp[p] && (k++ % 3 != 2)) want.push_back(p);
    CHECK(got == want);
    CHECK(prime_sizes(10.0, 5, [](int64_t p) { return p > 13 ? -7 : 1; }, got) == -7);
    CHECK(got.size() == 2 && got[0] == 11 && got[1] == 13);
    // L_max at c = 2, gamma = 1/2 is ceil(2 ln(2 |I|))
    for (int64_t n : {1, 2, 17, 1000, 65536, 1 << 20}) CHECK(lmax_rule(n, 2.0, 0.5) == (int64_t)std::ceil(2.0 * std::log(2.0 * (double)n)));
    printf("ok primes\n");
}

static void print_streams() {
    const uint64_t seeds[] = {0ull, 1711051520ull, 0xFFFFFFFFFFFFFFFFull};
    for (uint64_t seed : seeds) {
        const uint64_t k = Rng::key(seed, {Rng::Z, 3, 1, 7});
        printf("key %llu %llu\n", (unsigned long long)seed, (unsigned long long)k);
        for (uint64_t c = 0; c < 4; ++c)
            printf("draw %llu %llu %llu %.17g\n", (unsigned long long)seed, (unsigned long long)c,
                   (unsigned long long)Rng::draw(k, c), Rng::uniform01(k, c));
        for (uint64_t M : {1ull, 2ull, 65537ull, 2147483647ull, 0x8000000000000001ull}) {
            uint64_t ctr = 0;
            const uint64_t v = Rng::uniform_int(k, &ctr, M);
            CHECK(v < M);
            printf("int %llu %llu %llu %llu\n", (unsigned long long)seed, (unsigned long long)M,
                   (unsigned long long)v, (unsigned long long)ctr);
        }
    }
    printf("ok streams\n");
}

static void check_cache() {
    // size classes: at least the request, at most 12.5 % plus 2 MiB above it, 2 MiB multiples above
    for (size_t b : {(size_t)1, (size_t)255, (size_t)256, (size_t)257, (size_t)1 << 21, ((size_t)1 << 21) + 1,
                     (size_t)3 << 30, ((size_t)5 << 30) + 12345}) {
        const size_t c = size_class(b);
        CHECK(c >= b);
        if (b > ((size_t)2 << 20)) CHECK(c % ((size_t)2 << 20) == 0 && c <= b + b / 8 + ((size_t)2 << 20));
        else CHECK((c & (c - 1)) == 0);
    }
    // random traffic against host memory: blocks handed out are never in the cache, idle bytes
    // match the blocks held and stay within the cap, every block is freed once in the end
    std::mt19937_64 g(11);
    BlockCache C;
    C.limit = 64 << 20;
    std::set<void*> live;
    std::vector<std::pair<void*, size_t>> held;
    for (int it = 0; it < 20000; ++it) {
        if (held.empty() || g() % 3 != 0) {
            const size_t want = (size_t)1 + g() % (8u << 20);
            const size_t c = size_class(want);
            void* p = nullptr;
            size_t block = 0;
            BlockCache::Find r = C.take(c, &p, &block);
            if (r == BlockCache::NEEDS_DRAIN) {
                C.drained();
                r = C.take(c, &p, &block);
                CHECK(r == BlockCache::HIT);
            }
            if (r == BlockCache::MISS) {
                p = malloc(c);
                block = c;
                CHECK(p != nullptr);
            }
            CHECK(block >= c && block <= c + c / 2);
            CHECK(live.insert(p).second);
            ((volatile char*)p)[block - 1] = 1;   // the whole block is usable
            held.push_back({p, block});
        } else {
            const size_t i = (size_t)(g() % held.size());
            auto [p, block] = held[i];
            held[i] = held.back();
            held.pop_back();
            live.erase(p);
            if (!C.give_back(p, block)) free(p);
        }
        size_t sum = 0;
        for (auto* m : {&C.ready, &C.pending})
            for (auto& kv : *m) {
                sum += kv.first;
                CHECK(!live.count(kv.second));
            }
        CHECK(sum == C.idle && (int64_t)C.idle <= C.limit);
    }
    for (auto& h : held) free(h.first);
    const size_t idle = C.idle;
    CHECK(C.release_all([](void* p, size_t) { free(p); }) == idle && C.idle == 0);
    printf("ok cache\n");
}

int main() {
    check_rows();
    check_primes();
    print_streams();
    check_cache();
    return 0;
}
