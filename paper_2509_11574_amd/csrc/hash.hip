// Voxel-block hash of the colourised TSDF (Sec. 3.2.1, "SDF fusion": the SDF and
// colour live in a global hash table of voxel blocks, following InfiniTAM).
//
// Blocks of 8^3 lattice points sit in planar pools (the point (lx, ly, lz) of pool
// block b at b*512 + lx + 8 (ly + 8 lz), so the 64 lanes of a wavefront stream one
// z-slice's 64 points); an open-addressing table with linear probing maps packed
// block coordinates to pool blocks.  Points of unallocated blocks read tsdf 1,
// weight 0, colour 0 -- what the dense lattice holds where fusion never wrote.
//
//   k_hash_fill      the table's keys to empty (reset)
//   k_hash_begin     one lane: remembers the allocated count, clears the visible count
//   k_hash_alloc     one lane per pixel: the blocks of its ray's points in the
//                    truncation band (binary32 decisions), inserted by compare-and-
//                    swap; a new key takes the next pool block
//   k_hash_init      this frame's new pool blocks: tsdf 1, weights 0, colour 0
//   k_hash_visible   allocated blocks whose lattice box projects into the image
//                    (conservative), appended to the visible list
//   k_hash_fuse      one 512-lane group per visible block (groups stride over the
//                    list): the dense fusion update of every point
//   k_hash_block_min the minimum tsdf of each allocated block
//   k_hash_raycast   the dense march over the region's box; a sample whose stencil
//                    lies in one block that is unallocated or all positive reads
//                    positive, so such samples are skipped
// The pool order depends on which lane inserts a key first; no value depends on it.
#include <cmath>

#include "gps_internal.h"
#include "launch.h"
#include "prof.h"
#include "sdf_common.h"

namespace gps {

constexpr int kHB = GPS_HASH_BLOCK;
constexpr int kHB3 = kHB * kHB * kHB;
constexpr unsigned long long kHashEmpty = GPS_HASH_EMPTY;
constexpr int kHashGrid = 2048;  // workgroups of the kernels that stride over blocks

struct HashDev {
    unsigned long long* keys;
    int* slots;
    unsigned long long* bkey;
    int* state;  // allocated, allocated before this frame, visible, status bits
    int* visible;
    float* bmin;
    float* tsdf;
    float* w;
    float* rgb;
    float* cw;
    unsigned int mask;  // n_buckets - 1
    int cap;
    size_t pool;  // cap * 512: stride of the colour planes
    int n[3];
    int nb[3];  // blocks per axis
    float origin[3], voxel;
};

__device__ __forceinline__ unsigned long long hash_key(int bx, int by, int bz)
{
    return (unsigned long long)bx | ((unsigned long long)by << 21) | ((unsigned long long)bz << 42);
}

__device__ __forceinline__ void hash_unkey(unsigned long long k, int b[3])
{
    b[0] = (int)(k & 0x1fffffull);
    b[1] = (int)((k >> 21) & 0x1fffffull);
    b[2] = (int)((k >> 42) & 0x1fffffull);
}

// Home bucket: the splitmix64 finaliser of the key.
__device__ __forceinline__ unsigned int hash_home(unsigned long long k, unsigned int mask)
{
    k ^= k >> 30;
    k *= 0xbf58476d1ce4e5b9ull;
    k ^= k >> 27;
    k *= 0x94d049bb133111ebull;
    k ^= k >> 31;
    return (unsigned int)k & mask;
}

// Pool block of a key, or -1 (not allocated, or allocated without room).
__device__ __forceinline__ int hash_find(const HashDev& h, unsigned long long key)
{
    unsigned int s = hash_home(key, h.mask);
    for (unsigned int p = 0; p <= h.mask; ++p) {
        const unsigned long long k = h.keys[s];
        if (k == key) {
            const int v = h.slots[s];
            return v < h.cap ? v : -1;
        }
        if (k == kHashEmpty) return -1;
        s = (s + 1) & h.mask;
    }
    return -1;
}

__device__ __forceinline__ void hash_insert(const HashDev& h, unsigned long long key)
{
    unsigned int s = hash_home(key, h.mask);
    for (unsigned int p = 0; p <= h.mask; ++p) {
        const unsigned long long k = __hip_atomic_load(h.keys + s, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if (k == key) return;
        if (k == kHashEmpty) {
            const unsigned long long old = atomicCAS(h.keys + s, kHashEmpty, key);
            if (old == kHashEmpty) {  // this lane inserted the key: it takes the next pool block
                const int b = atomicAdd(h.state + 0, 1);
                if (b < h.cap) {
                    h.slots[s] = b;
                    h.bkey[b] = key;
                } else {
                    h.slots[s] = -1;
                    atomicOr(h.state + 3, 1);
                }
                return;
            }
            if (old == key) return;
        }
        s = (s + 1) & h.mask;
    }
    atomicOr(h.state + 3, 2);
}

__global__ void __launch_bounds__(256) k_hash_fill(unsigned long long* __restrict__ keys, unsigned int n,
                                                   int* __restrict__ state)
{
    const unsigned int i = blockIdx.x * 256u + threadIdx.x;
    if (i < n) keys[i] = kHashEmpty;
    if (i < 4) state[i] = 0;
}

__global__ void __launch_bounds__(64) k_hash_begin(int* __restrict__ state)
{
    if (threadIdx.x == 0) {
        state[1] = state[0];
        state[2] = 0;
    }
}

// Allocation: lane per pixel, the 2K+1 band points of its ray (the reference's
// orc_alloc_blocks takes the same binary32 steps).  Neighbouring pixels mostly
// reach the same blocks at the same band point, so a lane leaves a key to the lane
// before it in the wavefront when that lane has the same key at the same point (the
// first lane of such a run inserts it); every lane stays in the loop for the
// exchange, with an empty key where it has none.
__global__ void __launch_bounds__(256) k_hash_alloc(HashDev h, DevCam c, const float* __restrict__ depth, int K)
{
    const int p = blockIdx.x * 256 + threadIdx.x;
    const bool in = p < c.W * c.H;
    const float d = in ? depth[p] : 0.0f;
    const bool valid = in && d > 0.0f;
    const int i = in ? p % c.W : 0, j = in ? p / c.W : 0;
    const int lane = threadIdx.x & 63;
    float xn, yn, bsz;
    {
#pragma clang fp contract(off)
        xn = (float)i - c.cx;
        xn = xn / c.fx;
        yn = (float)j - c.cy;
        yn = yn / c.fy;
        bsz = h.voxel * (float)kHB;
    }
    unsigned long long last = kHashEmpty;
    for (int k = -K; k <= K; ++k) {
        int b[3];
        bool ok = valid;
        {
#pragma clang fp contract(off)
            float dz = (float)k * h.voxel;
            float z = d + dz;
            if (!(z > 0.0f)) ok = false;
            float xc = xn * z;
            float yc = yn * z;
            float q0 = xc - c.t[0];
            float q1 = yc - c.t[1];
            float q2 = z - c.t[2];
#pragma unroll
            for (int a = 0; a < 3; ++a) {
                float s = c.R[0 * 3 + a] * q0;
                float u = c.R[1 * 3 + a] * q1;
                s = s + u;
                float w = c.R[2 * 3 + a] * q2;
                s = s + w;
                float r = s - h.origin[a];
                r = r / bsz;
                float f = floorf(r);
                if (!(f >= 0.0f && f < (float)h.nb[a])) ok = false;
                b[a] = ok ? (int)f : 0;
            }
        }
        const unsigned long long key = ok ? hash_key(b[0], b[1], b[2]) : kHashEmpty;
        const unsigned long long left = __shfl_up(key, 1, 64);
        if (key == kHashEmpty || key == last || (lane > 0 && left == key)) continue;
        last = key;
        hash_insert(h, key);
    }
}

__global__ void __launch_bounds__(256) k_hash_init(HashDev h)
{
    const int lo = min(h.state[1], h.cap), hi = min(h.state[0], h.cap);
    for (int b = lo + (int)blockIdx.x; b < hi; b += (int)gridDim.x)
        for (int t = threadIdx.x; t < kHB3; t += 256) {
            const size_t v = (size_t)b * kHB3 + t;
            h.tsdf[v] = 1.0f;
            h.w[v] = 0.0f;
            h.rgb[v] = 0.0f;
            h.rgb[h.pool + v] = 0.0f;
            h.rgb[2 * h.pool + v] = 0.0f;
            h.cw[v] = 0.0f;
        }
}

// Visible list: a block whose eight corner points (of its lattice points) are all
// more than 1 mm behind the camera is out; one with a corner within 1 mm of the
// camera plane or behind it is in; otherwise it is in when the bounding box of the
// projected corners, grown by a pixel, meets the image (the projection of a box in
// front of the camera lies in the hull of its projected corners).
__global__ void __launch_bounds__(256) k_hash_visible(HashDev h, DevCam c)
{
    const int n = min(h.state[0], h.cap);
    for (int b = blockIdx.x * 256 + threadIdx.x; b < n; b += gridDim.x * 256) {
        int bc[3];
        hash_unkey(h.bkey[b], bc);
        float lo[3], hi[3];
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            const int x0 = bc[a] * kHB, x1 = min(bc[a] * kHB + kHB - 1, h.n[a] - 1);
            lo[a] = h.origin[a] + h.voxel * (float)x0;
            hi[a] = h.origin[a] + h.voxel * (float)x1;
        }
        int behind = 0, near_plane = 0;
        float umin = INFINITY, umax = -INFINITY, vmin = INFINITY, vmax = -INFINITY;
#pragma unroll
        for (int q = 0; q < 8; ++q) {
            const float p0 = (q & 1) ? hi[0] : lo[0], p1 = (q & 2) ? hi[1] : lo[1], p2 = (q & 4) ? hi[2] : lo[2];
            const float x = c.R[0] * p0 + c.R[1] * p1 + c.R[2] * p2 + c.t[0];
            const float y = c.R[3] * p0 + c.R[4] * p1 + c.R[5] * p2 + c.t[1];
            const float z = c.R[6] * p0 + c.R[7] * p1 + c.R[8] * p2 + c.t[2];
            if (z < -1e-3f) ++behind;
            if (z <= 1e-3f) {
                ++near_plane;
                continue;
            }
            const float u = c.fx * x / z + c.cx, v = c.fy * y / z + c.cy;
            umin = fminf(umin, u);
            umax = fmaxf(umax, u);
            vmin = fminf(vmin, v);
            vmax = fmaxf(vmax, v);
        }
        bool vis;
        if (behind == 8) vis = false;
        else if (near_plane > 0) vis = true;
        else vis = umax >= -1.5f && umin <= (float)c.W + 0.5f && vmax >= -1.5f && vmin <= (float)c.H + 0.5f;
        if (vis) h.visible[atomicAdd(h.state + 2, 1)] = b;
    }
}

__global__ void __launch_bounds__(kHB3) k_hash_fuse(HashDev h, FuseCtx ctx)
{
    const int nv = h.state[2];
    const int t = threadIdx.x;
    const int lx = t & 7, ly = (t >> 3) & 7, lz = t >> 6;
    for (int e = blockIdx.x; e < nv; e += gridDim.x) {
        const int b = h.visible[e];
        int bc[3];
        hash_unkey(h.bkey[b], bc);
        const int x = bc[0] * kHB + lx, y = bc[1] * kHB + ly, z = bc[2] * kHB + lz;
        if (x < h.n[0] && y < h.n[1] && z < h.n[2])
            fuse_point(ctx, x, y, z, (size_t)b * kHB3 + t, h.pool, h.tsdf, h.w, h.rgb, h.cw);
    }
}

__global__ void __launch_bounds__(256) k_hash_block_min(HashDev h)
{
    const int n = min(h.state[0], h.cap);
    const int lane = threadIdx.x & 63;
    for (int b = blockIdx.x * 4 + (threadIdx.x >> 6); b < n; b += gridDim.x * 4) {
        float m = INFINITY;
        for (int t = lane; t < kHB3; t += 64) m = fminf(m, h.tsdf[(size_t)b * kHB3 + t]);
        m = -wave_max(-m);
        if (lane == 0) h.bmin[b] = m;
    }
}

// The hashed volume as a Field of the march.  Successive samples of a ray mostly
// stay in one block, so the last lookup (key and pool block) is kept per lane; the
// table does not change during a raycast, so the kept answer is the table's.
// Per view and 16x16-pixel tile: the camera depths (lo, hi) outside which the
// view's rays read positive; tile t of view v at tile_base[v] + t.
struct HashRange {
    float2* range;  // null: no ranges
    int tile_base[GPS_MAX_VIEWS];
    int tiles_x[GPS_MAX_VIEWS];
};

struct HashField {
    HashDev h;
    const float2* range = nullptr;  // this view's tiles, or null
    int tiles_x = 0;
    mutable unsigned long long ckey = kHashEmpty, ckey2 = kHashEmpty;  // the last two lookups
    mutable int cblk = -1, cblk2 = -1;

    __device__ __forceinline__ bool depth_range(int, int col, int row, float* zlo, float* zhi) const
    {
        if (!range) return false;
        const float2 r = range[(row / GPS_HASH_TILE) * tiles_x + col / GPS_HASH_TILE];
        *zlo = r.x;
        *zhi = r.y;
        return true;
    }

    __device__ __forceinline__ int block_of(int bx, int by, int bz) const
    {
        const unsigned long long key = hash_key(bx, by, bz);
        if (key == ckey) return cblk;
        const unsigned long long k2 = ckey;
        const int b2 = cblk;
        ckey = key;
        cblk = key == ckey2 ? cblk2 : hash_find(h, key);
        ckey2 = k2;
        cblk2 = b2;
        return cblk;
    }

    __device__ __forceinline__ void fetch8(int plane, const int b[3], float q[8]) const
    {
        const float* f = plane == 0 ? h.tsdf : h.rgb + (size_t)(plane - 1) * h.pool;
        const float dflt = plane == 0 ? 1.0f : 0.0f;
        const int l0 = b[0] & 7, l1 = b[1] & 7, l2 = b[2] & 7;
        if (l0 < 7 && l1 < 7 && l2 < 7) {  // the stencil lies in one block
            const int blk = block_of(b[0] >> 3, b[1] >> 3, b[2] >> 3);
            if (blk < 0) {
#pragma unroll
                for (int k = 0; k < 8; ++k) q[k] = dflt;
                return;
            }
            const float* p = f + (size_t)blk * kHB3 + l0 + kHB * (l1 + kHB * l2);
            q[0] = p[0];
            q[1] = p[1];
            q[2] = p[kHB];
            q[3] = p[kHB + 1];
            q[4] = p[kHB * kHB];
            q[5] = p[kHB * kHB + 1];
            q[6] = p[kHB * kHB + kHB];
            q[7] = p[kHB * kHB + kHB + 1];
            return;
        }
        // The stencil crosses into the next block along the axes where its base sits at
        // local position 7: each block it touches is looked up once (through the kept
        // lookups: the next samples of the ray mostly read the same two blocks).
        const int B0 = b[0] >> 3, B1 = b[1] >> 3, B2 = b[2] >> 3;
        const bool cx = l0 == 7, cy = l1 == 7, cz = l2 == 7;
        auto find = [&](bool use, int dx, int dy, int dz) { return use ? block_of(B0 + dx, B1 + dy, B2 + dz) : -1; };
        const int bl0 = block_of(B0, B1, B2);
        const int bl1 = find(cx, 1, 0, 0), bl2 = find(cy, 0, 1, 0), bl3 = find(cx && cy, 1, 1, 0);
        const int bl4 = find(cz, 0, 0, 1), bl5 = find(cx && cz, 1, 0, 1), bl6 = find(cy && cz, 0, 1, 1);
        const int bl7 = find(cx && cy && cz, 1, 1, 1);
#pragma unroll
        for (int k = 0; k < 8; ++k) {
            const int x = b[0] + (k & 1), y = b[1] + ((k >> 1) & 1), z = b[2] + (k >> 2);
            const bool sx = (k & 1) && cx, sy = (k & 2) && cy, sz = (k & 4) && cz;
            const int blk = sz ? (sy ? (sx ? bl7 : bl6) : (sx ? bl5 : bl4)) : (sy ? (sx ? bl3 : bl2) : (sx ? bl1 : bl0));
            q[k] = blk < 0 ? dflt : f[(size_t)blk * kHB3 + (x & 7) + kHB * ((y & 7) + kHB * (z & 7))];
        }
    }

    // Samples based at local positions 0..6 of a block have their whole stencil in it:
    // positive when the block is unallocated or its minimum is positive.
    __device__ __forceinline__ bool skip_box(const int b[3], float lo[3], float hi[3]) const
    {
        if ((b[0] & 7) == 7 || (b[1] & 7) == 7 || (b[2] & 7) == 7) return false;
        const int blk = block_of(b[0] >> 3, b[1] >> 3, b[2] >> 3);
        if (blk >= 0 && !(h.bmin && h.bmin[blk] > kBrickPositive)) return false;
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            lo[k] = (float)((b[k] >> 3) * kHB);
            hi[k] = lo[k] + (float)(kHB - 1);
        }
        return true;
    }
};

// Depth ranges of the raycast: per view and tile, (lo, hi) start empty (+inf, 0).
__global__ void __launch_bounds__(256) k_hash_range_clear(float2* __restrict__ range, int n)
{
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i < n) range[i] = make_float2(INFINITY, 0.0f);
}

// One lane per (allocated block, view): the block's lattice box grown by one voxel
// on every side (it holds every sample whose stencil touches the block), clipped to
// the half-space of camera depths at least z_near (no sample lies nearer), is
// projected: the clipped box is the hull of its corners in the half-space and of the
// points where its edges cross the plane, so every tile that the bounding rectangle
// of their projections, grown by a pixel, meets takes the clipped box's depth range
// (depth is linear, so its extremes lie at those points).  With z_near below 1 mm a
// box reaching the camera plane covers every tile from depth 0.  Depths are
// positive, so their bit patterns order as the values do and integer atomics take
// the min and max.
__global__ void __launch_bounds__(256) k_hash_range(HashDev h, MarchArgs a, HashRange hr)
{
    const int n = min(h.state[0], h.cap);
    const int view = blockIdx.y;
    const DevCam& c = a.cams[view];
    const int tx = hr.tiles_x[view], ty = (c.H + GPS_HASH_TILE - 1) / GPS_HASH_TILE;
    unsigned int* rg = reinterpret_cast<unsigned int*>(hr.range + hr.tile_base[view]);
    const float zc = a.z_near * (1.0f - 1e-4f) - 1e-6f;  // the clipping plane, a little nearer than z_near
    for (int b = blockIdx.x * 256 + threadIdx.x; b < n; b += gridDim.x * 256) {
        int bc[3];
        hash_unkey(h.bkey[b], bc);
        float lo[3], hi[3];
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            lo[k] = h.origin[k] + h.voxel * (float)(bc[k] * kHB - 1);
            hi[k] = h.origin[k] + h.voxel * (float)(min(bc[k] * kHB + kHB - 1, h.n[k] - 1) + 1);
        }
        float X[8], Y[8], Z[8];
        float zmin = INFINITY, zmax = -INFINITY;
#pragma unroll
        for (int q = 0; q < 8; ++q) {
            const float p0 = (q & 1) ? hi[0] : lo[0], p1 = (q & 2) ? hi[1] : lo[1], p2 = (q & 4) ? hi[2] : lo[2];
            X[q] = c.R[0] * p0 + c.R[1] * p1 + c.R[2] * p2 + c.t[0];
            Y[q] = c.R[3] * p0 + c.R[4] * p1 + c.R[5] * p2 + c.t[1];
            Z[q] = c.R[6] * p0 + c.R[7] * p1 + c.R[8] * p2 + c.t[2];
            zmin = fminf(zmin, Z[q]);
            zmax = fmaxf(zmax, Z[q]);
        }
        if (!(zmax >= zc)) continue;  // wholly nearer than any sample
        int t0x, t1x, t0y, t1y;
        if (zmin < zc && zc < 1e-3f) {
            zmin = 0.0f;
            t0x = 0;
            t1x = tx - 1;
            t0y = 0;
            t1y = ty - 1;
        } else {
            float umin = INFINITY, umax = -INFINITY, vmin = INFINITY, vmax = -INFINITY;
            auto take = [&](float x, float y, float z) {
                const float u = c.fx * x / z + c.cx, v = c.fy * y / z + c.cy;
                umin = fminf(umin, u);
                umax = fmaxf(umax, u);
                vmin = fminf(vmin, v);
                vmax = fmaxf(vmax, v);
            };
#pragma unroll
            for (int q = 0; q < 8; ++q) {
                if (Z[q] >= zc) take(X[q], Y[q], Z[q]);
#pragma unroll
                for (int bit = 1; bit < 8; bit <<= 1) {
                    if (q & bit) continue;
                    const int r = q | bit;  // the edge (q, r)
                    if ((Z[q] < zc) != (Z[r] < zc)) {
                        const float t = (zc - Z[q]) / (Z[r] - Z[q]);
                        take(X[q] + t * (X[r] - X[q]), Y[q] + t * (Y[r] - Y[q]), zc);
                    }
                }
            }
            zmin = fmaxf(zmin, zc);
            if (!(umax >= -1.0f && umin <= (float)c.W && vmax >= -1.0f && vmin <= (float)c.H)) continue;
            // clamped to the view's tiles before the conversion (an empty range stays empty)
            const float T = (float)GPS_HASH_TILE;
            t0x = (int)fminf(fmaxf(floorf((umin - 1.0f) / T), 0.0f), (float)tx);
            t1x = (int)fmaxf(fminf(floorf((umax + 1.0f) / T), (float)(tx - 1)), -1.0f);
            t0y = (int)fminf(fmaxf(floorf((vmin - 1.0f) / T), 0.0f), (float)ty);
            t1y = (int)fmaxf(fminf(floorf((vmax + 1.0f) / T), (float)(ty - 1)), -1.0f);
        }
        // a little wider than the exact range: the rounding of the projection
        const unsigned int blo = __float_as_uint(fmaxf(zmin - 1e-4f * fabsf(zmin) - 1e-6f, 0.0f));
        const unsigned int bhi = __float_as_uint(zmax + 1e-4f * zmax + 1e-6f);
        for (int yy = t0y; yy <= t1y; ++yy)
            for (int xx = t0x; xx <= t1x; ++xx) {
                atomicMin(rg + 2 * (yy * tx + xx), blo);
                atomicMax(rg + 2 * (yy * tx + xx) + 1, bhi);
            }
    }
}

__global__ void __launch_bounds__(256) k_hash_raycast(MarchArgs a, HashDev h, HashRange hr)
{
    const int view = blockIdx.z;
    const DevCam& c = a.cams[view];
    const int col = blockIdx.x * 16 + (threadIdx.x & 15);
    const int row = blockIdx.y * 16 + (threadIdx.x >> 4);
    if (col >= c.W || row >= c.H) return;
    HashField f;  // this lane's field: it carries the lane's last lookup
    f.h = h;
    if (hr.range) {
        f.range = hr.range + hr.tile_base[view];
        f.tiles_x = hr.tiles_x[view];
    }
    march_pixel(a, f, view, col, row);
}

// ------------------------------------------------------------------ launches
static HashDev hash_dev(const gps_hash_volume& v)
{
    HashDev h;
    h.keys = reinterpret_cast<unsigned long long*>(v.keys);
    h.slots = v.slots;
    h.bkey = reinterpret_cast<unsigned long long*>(v.block_key);
    h.state = v.state;
    h.visible = v.visible;
    h.bmin = v.block_min;
    h.tsdf = v.tsdf;
    h.w = v.weight;
    h.rgb = v.rgb;
    h.cw = v.rgb_weight;
    h.mask = (unsigned int)v.n_buckets - 1u;
    h.cap = v.capacity;
    h.pool = (size_t)v.capacity * kHB3;
    h.n[0] = v.nx;
    h.n[1] = v.ny;
    h.n[2] = v.nz;
    h.nb[0] = (v.nx + kHB - 1) / kHB;
    h.nb[1] = (v.ny + kHB - 1) / kHB;
    h.nb[2] = (v.nz + kHB - 1) / kHB;
    for (int k = 0; k < 3; ++k) h.origin[k] = v.origin[k];
    h.voxel = v.voxel;
    return h;
}

gps_status launch_hash_reset(const gps_hash_volume* v, hipStream_t s)
{
    const unsigned int n = (unsigned int)v->n_buckets;
    GPS_LAUNCH(K_HASH, s, k_hash_fill, dim3((n + 255u) / 256u), dim3(256), 0, s,
               reinterpret_cast<unsigned long long*>(v->keys), n, v->state);
    return hipGetLastError() == hipSuccess ? GPS_OK : GPS_ERR_HIP;
}

gps_status launch_hash_fuse(const gps_hash_volume* v, const gps_camera* cam, const float* depth, const float* rgb,
                            hipStream_t s)
{
    HashDev h = hash_dev(*v);
    const DevCam c = dev_cam(*cam);
    // band points per side: ceil(mu / voxel), as the reference computes it
    const int K = (int)std::ceil((double)v->trunc / (double)v->voxel);
    FuseCtx ctx;
    ctx.ox = v->origin[0];
    ctx.oy = v->origin[1];
    ctx.oz = v->origin[2];
    ctx.voxel = v->voxel;
    ctx.mu = v->trunc;
    ctx.wmax = v->max_weight;
    ctx.cam = c;
    ctx.depth = depth;
    ctx.img = rgb;
    const int grid = v->capacity < kHashGrid ? v->capacity : kHashGrid;
    const unsigned int npx = (unsigned int)cam->width * (unsigned int)cam->height;
    GPS_LAUNCH(K_HASH, s, k_hash_begin, dim3(1), dim3(64), 0, s, v->state);
    GPS_LAUNCH(K_HASH, s, k_hash_alloc, dim3((npx + 255u) / 256u), dim3(256), 0, s, h, c, depth, K);
    GPS_LAUNCH(K_HASH, s, k_hash_init, dim3(grid), dim3(256), 0, s, h);
    const int vis_lanes = v->capacity < (1 << 16) ? v->capacity : (1 << 16);
    GPS_LAUNCH(K_HASH, s, k_hash_visible, dim3((vis_lanes + 255) / 256), dim3(256), 0, s, h, c);
    GPS_LAUNCH(K_FUSE, s, k_hash_fuse, dim3(grid), dim3(kHB3), 0, s, h, ctx);
    return hipGetLastError() == hipSuccess ? GPS_OK : GPS_ERR_HIP;
}

size_t hash_range_floats(const gps_camera* cams, int n_views)
{
    size_t n = 0;
    for (int v = 0; v < n_views; ++v) n += GPS_HASH_RANGE_FLOATS((size_t)cams[v].width, (size_t)cams[v].height);
    return n;
}

gps_status launch_hash_raycast(const gps_hash_volume* v, const gps_camera* cams, int n_views,
                               float* const* out_depth, float* const* out_rgb, float z_near, float step, float* range,
                               hipStream_t s)
{
    MarchArgs a;
    int maxW, maxH;
    march_setup(&a, v->nx, v->ny, v->nz, v->origin, v->voxel, z_near, step, cams, n_views, out_depth, out_rgb, &maxW,
                &maxH);
    const HashDev h = hash_dev(*v);
    const int bgrid = v->capacity < kHashGrid ? v->capacity : kHashGrid;
    if (v->block_min) GPS_LAUNCH(K_BRICK_MIN, s, k_hash_block_min, dim3((bgrid + 3) / 4), dim3(256), 0, s, h);
    HashRange hr;
    hr.range = nullptr;
    if (range) {
        int tiles = 0;
        for (int k = 0; k < n_views; ++k) {
            hr.tile_base[k] = tiles;
            hr.tiles_x[k] = (cams[k].width + GPS_HASH_TILE - 1) / GPS_HASH_TILE;
            tiles += hr.tiles_x[k] * ((cams[k].height + GPS_HASH_TILE - 1) / GPS_HASH_TILE);
        }
        hr.range = reinterpret_cast<float2*>(range);
        GPS_LAUNCH(K_RAYCAST, s, k_hash_range_clear, dim3((tiles + 255) / 256), dim3(256), 0, s, hr.range, tiles);
        const int lanes = v->capacity < (1 << 16) ? v->capacity : (1 << 16);
        GPS_LAUNCH(K_RAYCAST, s, k_hash_range, dim3((lanes + 255) / 256, n_views), dim3(256), 0, s, h, a, hr);
    }
    dim3 grid((maxW + 15) / 16, (maxH + 15) / 16, n_views);
    GPS_LAUNCH(K_RAYCAST, s, k_hash_raycast, grid, dim3(256), 0, s, a, h, hr);
    return hipGetLastError() == hipSuccess ? GPS_OK : GPS_ERR_HIP;
}

}  // namespace gps
