// Device building blocks for exact top-k selection fused into the scan.
//
// Ordering: a candidate is the pair (d, row) with d = the sum (or 65535 -
// sum when the largest sums are wanted) and row its index; pairs compare by d,
// then by row.  The k smallest pairs are the answer.
//
// A workgroup keeps, for each of its queries, a buffer of candidate keys in
// LDS and an exclusive bound on d: only rows with d < bound are appended.
// When a buffer may overflow, one wave prunes it: it finds T, the k-th
// smallest d in the buffer, by a 16-step bit descent over d (each step counts
// the keys below a trial value with one ballot per key slot), keeps every key
// with d <= T and lowers the bound to T.  Keys equal to T are all kept at that
// point; rows seen later have larger indices, so a later row with d == T can
// never beat them and the strict bound is exact.  The final selection trims
// the ties at T to the lowest row indices by a second descent over the row
// bits.  All of this is exact for any input, including massive ties.
#pragma once

#include "common.hpp"

namespace bolt {

// Local key of a candidate inside a row block of at most 65536 rows.
__device__ __forceinline__ uint32_t local_key(uint32_t d, uint32_t local_row) { return (d << 16) | local_row; }

// Population count of a wave ballot (wave-uniform).
__device__ __forceinline__ uint32_t ballot_count(bool p) { return (uint32_t)__popcll(__ballot(p)); }

// Number of lanes below this one whose predicate holds.
__device__ __forceinline__ uint32_t ballot_rank(bool p)
{
    const uint64_t m = __ballot(p);
    const uint32_t lo = __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u);
    return __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), lo);
}

struct PruneResult {
    uint32_t T;      // k-th smallest d (0x10000 if the buffer was left alone)
    uint32_t count;  // keys left in the buffer
};

// Wave-level prune of one query's buffer of local keys; the calling wave must
// be the only one touching the buffer.  `n` is the current fill.  Keeps every
// key with d <= T, T the k-th smallest d; with `exact`, ties at T are trimmed
// to the lowest rows so that exactly k keys remain.  The caller stores the
// returned count and lowers its bound to T.  Wave-uniform result.
template <int CAP>
__device__ PruneResult prune_local_lds(uint32_t *keys, uint32_t n, uint32_t k, bool exact)
{
    // Keys stay in LDS and are re-read at every descent step: for kernels
    // whose scan loop is register-bound, holding CAP/64 keys per lane in
    // registers would cost occupancy.
    constexpr int PER = (CAP + 63) / 64;
    const int lane = threadIdx.x & 63;
    if (n <= k)
        return {0x10000u, n};
    auto d_at = [&](int j) -> uint32_t {
        const uint32_t slot = (uint32_t)(lane + 64 * j);
        return slot < n ? (keys[slot] >> 16) : 0x10000u;   // 0x10000: never below a 16-bit trial
    };
    // T = largest t with #(d < t) < k, i.e. the k-th smallest d
    uint32_t T = 0;
    for (int b = 15; b >= 0; --b) {
        const uint32_t t = T | (1u << b);
        uint32_t c = 0;
#pragma unroll 4
        for (int j = 0; j < PER; ++j)
            c += ballot_count(d_at(j) < t);
        if (c < k)
            T = t;
    }
    uint32_t keep_row_max = 0xFFFFu;   // among ties at T, rows <= this are kept
    if (exact) {
        uint32_t lt = 0;
#pragma unroll 4
        for (int j = 0; j < PER; ++j)
            lt += ballot_count(d_at(j) < T);
        const uint32_t need = k - lt;   // >= 1
        uint32_t R = 0;                  // the need-th smallest row among ties at T
        for (int b = 15; b >= 0; --b) {
            const uint32_t t = R | (1u << b);
            uint32_t c = 0;
#pragma unroll 4
            for (int j = 0; j < PER; ++j) {
                const uint32_t slot = (uint32_t)(lane + 64 * j);
                const uint32_t key = slot < n ? keys[slot] : 0xFFFFFFFFu;
                c += ballot_count(slot < n && (key >> 16) == T && (key & 0xFFFFu) < t);
            }
            if (c < need)
                R = t;
        }
        keep_row_max = R;
    }
    // compaction: slots are read before being overwritten because the
    // destination index never exceeds the source index
    uint32_t base = 0;
#pragma unroll 1
    for (int j = 0; j < PER; ++j) {
        const uint32_t slot = (uint32_t)(lane + 64 * j);
        const uint32_t key = slot < n ? keys[slot] : 0xFFFFFFFFu;
        const uint32_t d = slot < n ? (key >> 16) : 0x10000u;
        const bool keep = d < T || (d == T && (key & 0xFFFFu) <= keep_row_max);
        const uint32_t r = ballot_rank(keep);
        const uint32_t total = ballot_count(keep);
        __builtin_amdgcn_wave_barrier();
        if (keep)
            keys[base + r] = key;
        base += total;
    }
    return {T, base};
}

// The same prune with the keys held in registers (CAP/64 per lane): faster,
// for kernels that can afford the registers.
template <int CAP>
__device__ PruneResult prune_local(uint32_t *keys, uint32_t n, uint32_t k, bool exact)
{
    constexpr int PER = (CAP + 63) / 64;
    const int lane = threadIdx.x & 63;
    if (n <= k)
        return {0x10000u, n};
    uint32_t key[PER];
    uint32_t d[PER];
#pragma unroll
    for (int j = 0; j < PER; ++j) {
        const uint32_t slot = (uint32_t)(lane + 64 * j);
        key[j] = slot < n ? keys[slot] : 0xFFFFFFFFu;
        d[j] = slot < n ? (key[j] >> 16) : 0x10000u;
    }
    uint32_t T = 0;
    for (int b = 15; b >= 0; --b) {
        const uint32_t t = T | (1u << b);
        uint32_t c = 0;
#pragma unroll
        for (int j = 0; j < PER; ++j)
            c += ballot_count(d[j] < t);
        if (c < k)
            T = t;
    }
    uint32_t keep_row_max = 0xFFFFu;
    if (exact) {
        uint32_t lt = 0;
#pragma unroll
        for (int j = 0; j < PER; ++j)
            lt += ballot_count(d[j] < T);
        const uint32_t need = k - lt;
        uint32_t R = 0;
        for (int b = 15; b >= 0; --b) {
            const uint32_t t = R | (1u << b);
            uint32_t c = 0;
#pragma unroll
            for (int j = 0; j < PER; ++j)
                c += ballot_count(d[j] == T && (key[j] & 0xFFFFu) < t);
            if (c < need)
                R = t;
        }
        keep_row_max = R;
    }
    uint32_t base = 0;
#pragma unroll
    for (int j = 0; j < PER; ++j) {
        const bool keep = d[j] < T || (d[j] == T && (key[j] & 0xFFFFu) <= keep_row_max);
        const uint32_t r = ballot_rank(keep);
        if (keep)
            keys[base + r] = key[j];
        base += ballot_count(keep);
    }
    return {T, base};
}

// Wave-level exact prune of a buffer of unique 48-bit keys (d << 32 | row):
// keeps exactly the k smallest.  Returns the k-th smallest key (or ~0 if the
// buffer held at most k keys); the caller stores count = min(n, k).
template <int CAP>
__device__ __attribute__((noinline)) uint64_t prune_u64(uint64_t *keys, uint32_t n, uint32_t k)
{
    constexpr int PER = (CAP + 63) / 64;
    const int lane = threadIdx.x & 63;
    if (n <= k)
        return ~0ull;
    uint64_t key[PER];
#pragma unroll
    for (int j = 0; j < PER; ++j) {
        const uint32_t slot = (uint32_t)(lane + 64 * j);
        key[j] = slot < n ? keys[slot] : ~0ull;
    }
    // Bits on which all n keys agree are the k-th smallest key's too: the
    // descent below runs only over the bits where they differ (the high bits
    // of d and the row bits above the largest row are common).
    uint64_t o = 0, a = ~0ull;
#pragma unroll
    for (int j = 0; j < PER; ++j)
        if ((uint32_t)(lane + 64 * j) < n) {
            o |= key[j];
            a &= key[j];
        }
#pragma unroll
    for (int m = 1; m < 64; m <<= 1) {
        const uint32_t olo = __shfl_xor((uint32_t)o, m), ohi = __shfl_xor((uint32_t)(o >> 32), m);
        const uint32_t alo = __shfl_xor((uint32_t)a, m), ahi = __shfl_xor((uint32_t)(a >> 32), m);
        o |= ((uint64_t)ohi << 32) | olo;
        a &= ((uint64_t)ahi << 32) | alo;
    }
    const uint64_t diff = o ^ a;   // nonzero for distinct keys (n > k >= 1)
    uint64_t ans = a;              // largest t with #(key < t) < k, i.e. the k-th smallest key
    if (diff) {
        const int hi = 63 - __builtin_clzll(diff), lo = __builtin_ctzll(diff);
        ans = a & ~((2ull << hi) - 1);
        for (int b = hi; b >= lo; --b) {
            const uint64_t t = ans | (1ull << b);
            uint32_t c = 0;
#pragma unroll
            for (int j = 0; j < PER; ++j)
                c += ballot_count(key[j] < t);
            if (c < k)
                ans = t;
        }
        ans |= a & ((1ull << lo) - 1);
    }
    uint32_t base = 0;
#pragma unroll
    for (int j = 0; j < PER; ++j) {
        const bool keep = key[j] <= ans;
        const uint32_t r = ballot_rank(keep);
        if (keep)
            keys[base + r] = key[j];
        base += ballot_count(keep);
    }
    (void)lane;
    return ans;
}

// prune_u64 over the smallest buffer size that holds n keys (up to CAP): the
// 48 counting passes cost in proportion to the registers each lane loads.
template <int CAP>
__device__ uint64_t prune_u64_fit(uint64_t *keys, uint32_t n, uint32_t k)
{
    if (CAP > 256 && n <= 256)
        return prune_u64<(CAP > 256 ? 256 : CAP)>(keys, n, k);
    if (CAP > 512 && n <= 512)
        return prune_u64<(CAP > 512 ? 512 : CAP)>(keys, n, k);
    if (CAP > 1024 && n <= 1024)
        return prune_u64<(CAP > 1024 ? 1024 : CAP)>(keys, n, k);
    return prune_u64<CAP>(keys, n, k);
}

}  // namespace bolt
