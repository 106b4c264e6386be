// Host-only logic of libmr1l that touches no GPU: the check that frequency rows are pairwise
// distinct (Alg. 2 input), the prime search and the lattice count of Alg. 1, the counter-based
// random streams of the method's draws, and the bookkeeping of the caching device allocator.
// Plain C++17 with no HIP dependency, so that it also builds with a host compiler alone (the
// library's sanitizer test compiles it with AddressSanitizer and UndefinedBehaviorSanitizer).
#pragma once

#include <stdint.h>

#include <algorithm>
#include <cmath>
#include <initializer_list>
#include <map>
#include <numeric>
#include <vector>

namespace mr1l {
namespace host {

// Rows a and b (a < b in input order) of f [n][d] that are equal, or false when all rows differ.
inline bool find_equal_rows(const int32_t* f, int64_t n, int d, int64_t* a, int64_t* b) {
    if (n < 2) return false;
    std::vector<int64_t> idx((size_t)n);
    std::iota(idx.begin(), idx.end(), 0);
    std::sort(idx.begin(), idx.end(), [&](int64_t x, int64_t y) {
        const bool lt = std::lexicographical_compare(f + x * d, f + x * d + d, f + y * d, f + y * d + d);
        const bool gt = std::lexicographical_compare(f + y * d, f + y * d + d, f + x * d, f + x * d + d);
        return lt || (!gt && x < y);   // equal rows keep their input order
    });
    for (int64_t i = 1; i < n; ++i)
        if (std::equal(f + idx[i - 1] * d, f + idx[i - 1] * d + d, f + idx[i] * d)) {
            *a = idx[i - 1];
            *b = idx[i];
            return true;
        }
    return false;
}

// Trial division (the lattice sizes of Alg. 1 stay below 2^31).
inline bool is_prime(int64_t p) {
    if (p < 2) return false;
    if (p % 2 == 0) return p == 2;
    for (int64_t q = 3; q * q <= p; q += 2)
        if (p % q == 0) return false;
    return true;
}

// L_max = ceil(c^2/(c-1)^2 (ln|I| - ln gamma) / 2)  (Alg. 1, first step)
inline int64_t lmax_rule(int64_t n, double c, double gamma) {
    return (int64_t)std::ceil(c * c / ((c - 1.0) * (c - 1.0)) * (std::log((double)n) - std::log(gamma)) / 2.0);
}

// The ``count`` smallest primes p > lambda for which ``injective(p)`` holds (the set P^I of Alg. 1:
// k -> k mod p injective on I).  ``injective`` returns 1 (yes), 0 (no) or a negative error code,
// which ends the search; the code is returned and ``out`` holds the primes found so far.
template <typename Injective>
int prime_sizes(double lambda, int64_t count, Injective&& injective, std::vector<int64_t>& out) {
    out.clear();
    for (int64_t p = (int64_t)std::floor(lambda) + 1; (int64_t)out.size() < count; ++p) {
        if (!is_prime(p)) continue;
        const int ok = injective(p);
        if (ok < 0) return ok;
        if (ok) out.push_back(p);
    }
    return 0;
}

// Counter-based SplitMix64 streams (published generator; the key derivation is this project's):
//   key(seed, f1..fm): k = seed; k = mix64(k + GAMMA (f + 1)) for each field f
//   draw(k, c) = mix64(k + GAMMA (c + 1))
struct Rng {
    static constexpr uint64_t GAMMA = 0x9E3779B97F4A7C15ull;
    static uint64_t mix64(uint64_t x) {
        x ^= x >> 30;
        x *= 0xBF58476D1CE4E5B9ull;
        x ^= x >> 27;
        x *= 0x94D049BB133111EBull;
        x ^= x >> 31;
        return x;
    }
    static uint64_t key(uint64_t seed, std::initializer_list<int64_t> fields) {
        uint64_t k = seed;
        for (int64_t f : fields) k = mix64(k + GAMMA * (uint64_t)(f + 1));
        return k;
    }
    static uint64_t draw(uint64_t k, uint64_t c) { return mix64(k + GAMMA * (c + 1)); }
    static double uniform01(uint64_t k, uint64_t c) { return (double)(draw(k, c) >> 11) * 0x1.0p-53; }
    // unbiased integer in [0, M): rejection of draws below 2^64 mod M; advances *c
    static uint64_t uniform_int(uint64_t k, uint64_t* c, uint64_t M) {
        const uint64_t floor_reject = (0 - M) % M;   // == 2^64 mod M
        for (;;) {
            const uint64_t u = draw(k, (*c)++);
            if (u >= floor_reject) return u % M;
        }
    }
    enum Purpose : int64_t { Z = 1, ANCHOR1D = 2, ANCHOR = 3, NOISE = 4, ZREDRAW = 5 };
};

// ---- caching allocator bookkeeping -----------------------------------------------------------------
// Size classes: powers of two from 256 B up to 2 MiB; above, eight classes per octave rounded up
// to a multiple of 2 MiB (at most 12.5 % slack plus the rounding).
inline size_t size_class(size_t b) {
    constexpr size_t kMiB2 = (size_t)2 << 20;
    if (b <= kMiB2) {
        size_t c = 256;
        while (c < b) c <<= 1;
        return c;
    }
    int k = 0;
    while (k < 63 && ((size_t)1 << (k + 1)) <= b) ++k;   // 2^k <= b < 2^(k+1)
    const size_t step = ((size_t)1 << k) / 8;
    const size_t c = (b + step - 1) / step * step;
    return (c + kMiB2 - 1) / kMiB2 * kMiB2;
}

// Idle blocks of one device.  A freed block is "pending" (work queued before the free may still
// use it) until the owner reports a device-wide drain; only "ready" blocks are handed out.  Idle
// bytes (ready + pending) stay within ``limit``.  The owner holds its lock around every call and
// does the device calls (synchronise, free) itself.
struct BlockCache {
    std::multimap<size_t, void*> ready, pending;
    size_t idle = 0;
    int64_t limit = -1;   // -1 until the owner sets it

    enum Find { HIT, NEEDS_DRAIN, MISS };
    // a block of class c, or of a class at most 1.5 c: HIT (removed from the cache), NEEDS_DRAIN
    // (only a pending block fits: drain the device, call drained(), ask again) or MISS
    Find take(size_t c, void** p, size_t* block) {
        const size_t cmax = c + c / 2;
        auto fit = [&](std::multimap<size_t, void*>& m) {
            auto it = m.lower_bound(c);
            return (it != m.end() && it->first <= cmax) ? it : m.end();
        };
        auto it = fit(ready);
        if (it == ready.end()) return fit(pending) != pending.end() ? NEEDS_DRAIN : MISS;
        *p = it->second;
        *block = it->first;
        idle -= it->first;
        ready.erase(it);
        return HIT;
    }
    // the device has drained: every pending block is reusable
    void drained() {
        ready.insert(pending.begin(), pending.end());
        pending.clear();
    }
    // keep a freed block of size c (true) or, beyond the cap, leave it to the owner to free (false)
    bool give_back(void* p, size_t c) {
        if (limit < 0 || (int64_t)(idle + c) > limit) return false;
        pending.insert({c, p});
        idle += c;
        return true;
    }
    // every idle block, handed to free_block(ptr, size); returns the bytes released
    template <typename FreeBlock>
    size_t release_all(FreeBlock&& free_block) {
        size_t freed = 0;
        for (auto* m : {&ready, &pending}) {
            for (auto& kv : *m) {
                free_block(kv.second, kv.first);
                freed += kv.first;
            }
            m->clear();
        }
        idle = 0;
        return freed;
    }
};

}  // namespace host
}  // namespace mr1l
