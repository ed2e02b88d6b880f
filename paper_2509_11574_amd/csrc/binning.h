// Tuning constants of the instance binning (expansion and per-tile counters).
// Kept apart from the headers of the compositing kernels, which they do not affect.
#pragma once

#include "gps_internal.h"

namespace gps {

constexpr int kExpG = 64;             // view-Gaussians per block of the instance expansion (kBlk lanes walk
                                      // their tile rectangles: about kBlk / kExpG lanes per Gaussian)
constexpr int kExpGLog2 = 6;
static_assert((1 << kExpGLog2) == kExpG && kBlk % kExpG == 0, "expansion share");
constexpr int kCntSplit = 4;          // sub-counters per tile for the count pass's atomics (block index mod 4):
                                      // fewer increments queue on one address
constexpr int kSmallSort = 512;       // one wavefront sorts up to this many keys in registers
// Tiles of at least kLongTile keys (exactly those whose queue bucket floor(log2(n + 1))
// is log2(kSmallSort) or more, so they lead the longest-first queue) take the block sort.
constexpr unsigned int kLongTile = kSmallSort - 1;


// Bitonic network in which every compare-exchange puts the smaller key at the
// lower index (the first step of each merge compares mirrored pairs: element e
// with e ^ (k - 1) inside its aligned block of k), so padding with +inf keys
// never moves into the sorted range.  wave_sort_regs sorts up to 64 R keys in
// registers of one wavefront: element e = 64 r + lane sits in register r of that
// lane, so a compare-exchange at distance < 64 is a lane exchange (shuffle) and
// one at distance >= 64 a swap between two registers of the same lane.  No LDS
// and no barriers.
__device__ __forceinline__ unsigned long long shfl_xor_u64(unsigned long long v, int m)
{
    const unsigned int lo = __shfl_xor((unsigned int)v, m, 64);
    const unsigned int hi = __shfl_xor((unsigned int)(v >> 32), m, 64);
    return ((unsigned long long)hi << 32) | lo;
}

__device__ __forceinline__ unsigned long long min_u64(unsigned long long a, unsigned long long b) { return a < b ? a : b; }
__device__ __forceinline__ unsigned long long max_u64(unsigned long long a, unsigned long long b) { return a < b ? b : a; }

// Sorts the n <= 64 R keys at key[0..n) ascending; one wavefront, lane `lane`.
template <int R>
__device__ __forceinline__ void wave_sort_regs(unsigned long long* key, int n, int lane)
{
    constexpr int P = 64 * R;
    unsigned long long x[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const int e = 64 * r + lane;
        x[r] = e < n ? key[e] : ~0ull;
    }
#pragma unroll
    for (int k = 2; k <= P; k <<= 1) {
        // mirrored step: e <-> e ^ (k - 1); e is the lower index when bit k/2 of e is clear
        if (k <= 64) {
#pragma unroll
            for (int r = 0; r < R; ++r) {
                const unsigned long long o = shfl_xor_u64(x[r], k - 1);
                x[r] = (lane & (k >> 1)) == 0 ? min_u64(x[r], o) : max_u64(x[r], o);
            }
        } else {
            const int jr = k / 64 - 1;  // partner: register r ^ jr of lane ^ 63
            unsigned long long o[R];
#pragma unroll
            for (int r = 0; r < R; ++r) o[r] = shfl_xor_u64(x[r ^ jr], 63);
#pragma unroll
            for (int r = 0; r < R; ++r)
                x[r] = ((64 * r) & (k >> 1)) == 0 ? min_u64(x[r], o[r]) : max_u64(x[r], o[r]);
        }
        // half-cleaner steps: e <-> e ^ j, j = k/4 .. 1
#pragma unroll
        for (int j = k >> 2; j > 0; j >>= 1) {
            if (j >= 64) {
                const int jr = j / 64;
#pragma unroll
                for (int r = 0; r < R; ++r) {
                    if ((r & jr) == 0) {
                        const unsigned long long a = x[r], b = x[r | jr];
                        x[r] = min_u64(a, b);
                        x[r | jr] = max_u64(a, b);
                    }
                }
            } else {
#pragma unroll
                for (int r = 0; r < R; ++r) {
                    const unsigned long long o = shfl_xor_u64(x[r], j);
                    x[r] = (lane & j) == 0 ? min_u64(x[r], o) : max_u64(x[r], o);
                }
            }
        }
    }
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const int e = 64 * r + lane;
        if (e < n) key[e] = x[r];
    }
}

// Sorts the n < kLongTile keys at key[0..n) with the smallest register network
// that holds them (one wavefront).
__device__ __forceinline__ void wave_sort_tile(unsigned long long* key, int n, int lane)
{
    if (n <= 64) wave_sort_regs<1>(key, n, lane);
    else if (n <= 128) wave_sort_regs<2>(key, n, lane);
    else if (n <= 256) wave_sort_regs<4>(key, n, lane);
    else wave_sort_regs<8>(key, n, lane);
}

}  // namespace gps
