// Voxelization with direct-light injection (Section 4.4 "Voxelization
// Process", Section 5.4.4 "Voxelization"): every triangle is rasterized once
// along its dominant axis onto an N x N viewport; every fragment (pixel centre
// inside the projected triangle) is the voxel (pixel, floor(depth)) and gets
// the Phong light of the surface point without its glossy term (ambient +
// diffuse with the triangle's own normal, distance attenuation) and alpha 1.
//
// Determinism: coverage and depth are decided on vertices snapped to 1/256
// voxel by exact integer edge functions and an exact floor division (a
// centre on an edge belongs to the triangle when the counter-clockwise edge
// runs upward or horizontally leftward, so shared edges are covered once);
// fragments falling into the same voxel are averaged through 64-bit
// fixed-point sums and a count, so the result does not depend on the order in
// which fragments arrive.
//
// Surface attributes (optional): per voxel the average of the fragments' unit
// triangle normals and of their triangle colours, through the same kind of
// fixed-point sums (a further 3D texture of surface normals is what more light
// bounces need, Section 6.2.2; deferred voxel cone tracing keeps albedo and
// normal textures from voxelization, Section 5.1.3).
//
// Launch: a setup pass (one thread per triangle) writes each triangle's
// rasterization record and the pixel count of its bounding box; a scan turns
// the counts into offsets (one workgroup for up to 4096 triangles, else three
// phases: sums of 1024 counts, one workgroup over those sums, offsets inside
// each 1024); the raster pass then walks the
// flattened pixel space, one lane per bounding-box pixel, each lane finding its
// triangle by a binary search of the offsets.  A wall-sized triangle spreads
// over many waves and a thousand one-pixel triangles fill a wave.
//
// Sparse accumulators: only voxels that a fragment reaches get one (most of a
// scene's grid is empty).  The output grids are zero-filled (base first;
// normal and albedo by workgroups of the raster launch of their own); while the
// raster pass runs, the alpha word of a reached voxel in `base` holds the
// index + 1 of its accumulator slot, taken from a counter by the first
// fragment to claim the voxel (a compare-and-swap to a claim mark, then the
// index is published; fragments that find the mark read the word again until
// the index appears, which follows the claim directly).  A slot is {int64
// r, g, b; uint32 count; uint32 voxel + 1} (32 bytes), and with surface
// attributes {int64 nx, ny, nz, r, g, b} (48 bytes) more.  Only as many slots
// as the triangles' bounding boxes hold pixels (at most one per voxel) are
// cleared, by fill kernels (no memset, so the path can be captured in a
// graph); the resolve pass walks the used slots and writes their voxels.
// Which slot a voxel gets depends on arrival order; the integer sums in it do
// not, so the grids are the same bits whatever the order.
#include "vct_internal.h"

namespace {

constexpr int kSub = 256;                 // subpixels per voxel
constexpr int kCoordLimit = 1 << 19;      // |snapped coordinate| bound of the exact arithmetic
constexpr float kFix = 4294967296.0f;     // 2^32: fixed-point scale of the colour sums
constexpr float kFixMax = 268435456.0f;   // 2^28: per-fragment colour bound of the fixed point

struct VoxArgs {
    int32_t n;
    float origin[3];
    float voxel;          // extent / N
    float snap_scale;     // 256 N / extent, float32
    int32_t n_lights;
    float light_pos[VCT_MAX_LIGHTS][3];
    float light_color[VCT_MAX_LIGHTS][3];
    float att[VCT_MAX_LIGHTS][3];
    float ambient, diffuse;
};

struct VoxAcc {
    unsigned long long r, g, b;
    unsigned int count, voxel;   // voxel: linear voxel index + 1 (0: slot unused)
};

constexpr unsigned int kClaimed = 0xffffffffu;   // alpha word of a voxel whose slot is being taken
constexpr int kMaxSpin = 1 << 24;                // bound of the wait for a claimed voxel's slot

struct SurfAcc {
    unsigned long long n[3], c[3];
};

// Zero the output grids (n float4 each; normal and albedo may be null) and the slot counter.
__global__ void k_clear(uint4* __restrict__ base, uint4* __restrict__ normal, uint4* __restrict__ albedo, size_t n,
                        unsigned int* __restrict__ counter) {
    const uint4 z = make_uint4(0u, 0u, 0u, 0u);
    if (blockIdx.x == 0 && threadIdx.x == 0) *counter = 0u;
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) {
        base[i] = z;
        if (normal) {
            normal[i] = z;
            albedo[i] = z;
        }
    }
}

// Zero the first min(*total, cap) slots: no more can be taken than there are
// bounding-box pixels (each fragment claims at most one voxel) or voxels.
__global__ void k_clear_slots(uint4* __restrict__ acc, uint4* __restrict__ surf, const unsigned long long* total_p,
                              unsigned long long cap) {
    const unsigned long long used = min(*total_p, cap);
    const uint4 z = make_uint4(0u, 0u, 0u, 0u);
    const size_t stride = (size_t)gridDim.x * blockDim.x;
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < used * 2; i += stride) acc[i] = z;
    if (surf)
        for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < used * 3; i += stride) surf[i] = z;
}

__device__ __forceinline__ long long floor_div(long long a, long long b) {   // b > 0
    long long q = a / b;
    return (a % b != 0 && a < 0) ? q - 1 : q;
}

__device__ __forceinline__ bool top_left(long long dx, long long dy) { return dy > 0 || (dy == 0 && dx < 0); }

__device__ __forceinline__ unsigned long long to_fixed(float v) {
    v = fminf(fmaxf(v, -kFixMax), kFixMax);
    return (unsigned long long)(long long)rintf(v * kFix);
}

// Rasterization setup of one triangle: snapped, swizzled vertices (counter-
// clockwise), plane coefficients, pixel bounding box, the unit normal of the
// original triangle and its colour.  npx = 0 when the triangle produces nothing.
struct TriSetup {
    long long A[3], B[3], C[3];      // (X2, Y2, W) subpixel coordinates
    long long nx, ny, nw;            // plane: nw W = nw A.w - nx (X - A.x) - ny (Y - A.y), nw > 0
    int32_t i0, j0, w, npx;          // bounding box origin and width in pixels, pixel count
    int32_t sx, sy, sw, pad;         // source axes of X2, Y2, W
    float n[3], col[3];
};

constexpr int kScanBlock = 1024;     // counts per block of the offset scan (256 threads x 4)
constexpr int kScanThreads = 1024;   // threads of the one-workgroup scan of block sums

__global__ __launch_bounds__(256) void k_tri_setup(VoxArgs a, const float* __restrict__ tris,
                                                   const float* __restrict__ colors, long long n_tris,
                                                   TriSetup* __restrict__ setup, unsigned long long* __restrict__ counts) {
    const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n_tris) return;
    TriSetup r{};
    counts[t] = 0;
    // snapped vertices (float32 arithmetic, round half to even)
    float vf[3][3];
    long long s[3][3];
    bool ok = true;
    for (int k = 0; k < 3; ++k)
        for (int i = 0; i < 3; ++i) {
            const float p = tris[t * 9 + k * 3 + i];
            vf[k][i] = p;
            const float u = rintf((p - a.origin[i]) * a.snap_scale);
            ok = ok && isfinite(p) && fabsf(u) <= (float)kCoordLimit;
            s[k][i] = ok ? (long long)u : 0;
        }
    if (!ok) {
        setup[t] = r;
        return;
    }
    // dominant axis of the snapped normal (ties to x, then y, then z)
    long long e1[3], e2[3];
    for (int i = 0; i < 3; ++i) {
        e1[i] = s[1][i] - s[0][i];
        e2[i] = s[2][i] - s[0][i];
    }
    const long long nrm[3] = {e1[1] * e2[2] - e1[2] * e2[1], e1[2] * e2[0] - e1[0] * e2[2],
                              e1[0] * e2[1] - e1[1] * e2[0]};
    const long long ax = nrm[0] < 0 ? -nrm[0] : nrm[0], ay = nrm[1] < 0 ? -nrm[1] : nrm[1],
                    az = nrm[2] < 0 ? -nrm[2] : nrm[2];
    const int dom = (ax >= ay && ax >= az) ? 0 : (ay >= az ? 1 : 2);
    // projection frame (X2, Y2 | W): x-dominant (z, y | x), y-dominant (x, z | y), z-dominant (x, y | z)
    r.sx = dom == 0 ? 2 : 0;
    r.sy = dom == 1 ? 2 : 1;
    r.sw = dom;
    for (int k = 0; k < 3; ++k) {
        long long* V = k == 0 ? r.A : (k == 1 ? r.B : r.C);
        V[0] = s[k][r.sx];
        V[1] = s[k][r.sy];
        V[2] = s[k][r.sw];
    }
    const long long area = (r.B[0] - r.A[0]) * (r.C[1] - r.A[1]) - (r.B[1] - r.A[1]) * (r.C[0] - r.A[0]);
    if (area == 0) {
        setup[t] = TriSetup{};
        return;
    }
    if (area < 0) {
        for (int i = 0; i < 3; ++i) {
            const long long tmp = r.B[i];
            r.B[i] = r.C[i];
            r.C[i] = tmp;
        }
    }
    const long long h = kSub / 2;
    const long long minx = min(r.A[0], min(r.B[0], r.C[0])), maxx = max(r.A[0], max(r.B[0], r.C[0]));
    const long long miny = min(r.A[1], min(r.B[1], r.C[1])), maxy = max(r.A[1], max(r.B[1], r.C[1]));
    const long long i0 = max(0ll, -floor_div(h - minx, kSub)), i1 = min((long long)a.n - 1, floor_div(maxx - h, kSub));
    const long long j0 = max(0ll, -floor_div(h - miny, kSub)), j1 = min((long long)a.n - 1, floor_div(maxy - h, kSub));
    if (i1 < i0 || j1 < j0) {
        setup[t] = TriSetup{};
        return;
    }
    const long long f1[3] = {r.B[0] - r.A[0], r.B[1] - r.A[1], r.B[2] - r.A[2]};
    const long long f2[3] = {r.C[0] - r.A[0], r.C[1] - r.A[1], r.C[2] - r.A[2]};
    r.nx = f1[1] * f2[2] - f1[2] * f2[1];
    r.ny = f1[2] * f2[0] - f1[0] * f2[2];
    r.nw = f1[0] * f2[1] - f1[1] * f2[0];
    r.i0 = (int32_t)i0;
    r.j0 = (int32_t)j0;
    r.w = (int32_t)(i1 - i0 + 1);
    r.npx = (int32_t)((i1 - i0 + 1) * (j1 - j0 + 1));
    // lighting: unit normal of the original triangle as wound
    const float d1[3] = {vf[1][0] - vf[0][0], vf[1][1] - vf[0][1], vf[1][2] - vf[0][2]};
    const float d2[3] = {vf[2][0] - vf[0][0], vf[2][1] - vf[0][1], vf[2][2] - vf[0][2]};
    float tn[3] = {d1[1] * d2[2] - d1[2] * d2[1], d1[2] * d2[0] - d1[0] * d2[2], d1[0] * d2[1] - d1[1] * d2[0]};
    const float l = sqrtf(tn[0] * tn[0] + tn[1] * tn[1] + tn[2] * tn[2]);
    const float il = l > 0.f ? 1.0f / l : 0.f;
    for (int i = 0; i < 3; ++i) {
        r.n[i] = tn[i] * il;
        r.col[i] = colors[t * 3 + i];
    }
    setup[t] = r;
    counts[t] = (unsigned long long)r.npx;
}

// Offset scan, phase 1: the sum of each block of kScanBlock counts.
__global__ __launch_bounds__(256) void k_block_sums(const unsigned long long* __restrict__ c, long long n,
                                                    unsigned long long* __restrict__ bsum) {
    __shared__ unsigned long long s[4];
    const long long i0 = (long long)blockIdx.x * kScanBlock + threadIdx.x * 4;
    unsigned long long v = 0;
#pragma unroll
    for (int k = 0; k < 4; ++k) v += i0 + k < n ? c[i0 + k] : 0ull;
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    if ((threadIdx.x & 63) == 0) s[threadIdx.x >> 6] = v;
    __syncthreads();
    if (threadIdx.x == 0) bsum[blockIdx.x] = (s[0] + s[1]) + (s[2] + s[3]);
}

// Phase 2, one workgroup: bsum[b] becomes the sum of bsum[0..b); *total the sum of all.
__global__ __launch_bounds__(kScanThreads) void k_scan_sums(unsigned long long* __restrict__ bsum, long long nb,
                                                            unsigned long long* __restrict__ total) {
    __shared__ unsigned long long s[kScanThreads];
    const long long per = (nb + kScanThreads - 1) / kScanThreads;
    const long long b = threadIdx.x * per, e = min(b + per, nb);
    unsigned long long own = 0;
    for (long long i = b; i < e; ++i) own += bsum[i];
    s[threadIdx.x] = own;
    __syncthreads();
    for (int off = 1; off < kScanThreads; off <<= 1) {   // inclusive Hillis-Steele scan
        const unsigned long long add = threadIdx.x >= (unsigned)off ? s[threadIdx.x - off] : 0ull;
        __syncthreads();
        s[threadIdx.x] += add;
        __syncthreads();
    }
    unsigned long long run = s[threadIdx.x] - own;
    for (long long i = b; i < e; ++i) {
        const unsigned long long c = bsum[i];
        bsum[i] = run;
        run += c;
    }
    if (threadIdx.x == kScanThreads - 1) *total = s[kScanThreads - 1];
}

// Phase 3: counts become exclusive offsets, in place (block base + prefix inside the block).
__global__ __launch_bounds__(256) void k_block_offsets(unsigned long long* __restrict__ c, long long n,
                                                       const unsigned long long* __restrict__ bsum) {
    __shared__ unsigned long long s[256];
    const long long i0 = (long long)blockIdx.x * kScanBlock + threadIdx.x * 4;
    unsigned long long v[4], own = 0;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        v[k] = i0 + k < n ? c[i0 + k] : 0ull;
        own += v[k];
    }
    s[threadIdx.x] = own;
    __syncthreads();
    for (int off = 1; off < 256; off <<= 1) {   // inclusive Hillis-Steele scan of the thread sums
        const unsigned long long add = threadIdx.x >= (unsigned)off ? s[threadIdx.x - off] : 0ull;
        __syncthreads();
        s[threadIdx.x] += add;
        __syncthreads();
    }
    unsigned long long run = bsum[blockIdx.x] + s[threadIdx.x] - own;
#pragma unroll
    for (int k = 0; k < 4; ++k)
        if (i0 + k < n) {
            c[i0 + k] = run;
            run += v[k];
        }
}

// The whole offset scan in one workgroup, for meshes of at most kScanSmall
// triangles (1024 threads x 4 counts): one launch in place of the three of
// the blocked scan, with the same integer sums.
constexpr int kScanSmall = 4096;
__global__ __launch_bounds__(1024) void k_scan_small(unsigned long long* __restrict__ c, long long n,
                                                     unsigned long long* __restrict__ total) {
    __shared__ unsigned long long s[1024];
    const long long i0 = (long long)threadIdx.x * 4;
    unsigned long long v[4], own = 0;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        v[k] = i0 + k < n ? c[i0 + k] : 0ull;
        own += v[k];
    }
    s[threadIdx.x] = own;
    __syncthreads();
    for (int off = 1; off < 1024; off <<= 1) {   // inclusive Hillis-Steele scan of the thread sums
        const unsigned long long add = threadIdx.x >= (unsigned)off ? s[threadIdx.x - off] : 0ull;
        __syncthreads();
        s[threadIdx.x] += add;
        __syncthreads();
    }
    unsigned long long run = s[threadIdx.x] - own;
#pragma unroll
    for (int k = 0; k < 4; ++k)
        if (i0 + k < n) {
            c[i0 + k] = run;
            run += v[k];
        }
    if (threadIdx.x == 1023) *total = s[1023];
}

// floor(a / b) for b > 0 from a float estimate corrected in exact int64 arithmetic
// (|a| < 2^63, quotients here are below 2^31).
__device__ __forceinline__ long long floor_div_est(long long a, long long b) {
    long long q = (long long)floorf((float)a / (float)b);
    while (q * b > a) --q;
    while ((q + 1) * b <= a) ++q;
    return q;
}

// One lane per bounding-box pixel of the flattened pixel space (triangle t
// owns [offs[t], offs[t] + npx)), in a grid-stride loop; a lane's triangle is
// the last t with offs[t] <= g (a triangle without pixels has offs[t] =
// offs[t + 1] and is passed over).
//
// With surface attributes the first kZeroBlocks workgroups instead zero the
// normal and albedo grids (n float4 each, walked as one index space), which
// nothing reads or writes before the resolve pass: their stores stream to HBM
// while the raster workgroups wait on their atomics.  (Cornell mesh at 256^3:
// 0.41 ms for the call with a separate fill, 0.33 ms with 256 such
// workgroups, 0.35 / 0.38 ms with 512 / 1024, 0.36 / 0.38 ms with 192 / 128.)
constexpr int kRasterBlocks = 2048;
constexpr int kZeroBlocks = 256;

template <bool SURF>
__global__ __launch_bounds__(256) void k_raster(VoxArgs a, const TriSetup* __restrict__ setup,
                                                const unsigned long long* __restrict__ offs, long long n_tris,
                                                const unsigned long long* __restrict__ total_p,
                                                VoxAcc* __restrict__ acc, SurfAcc* __restrict__ surf,
                                                unsigned int* __restrict__ base_words,
                                                unsigned int* __restrict__ counter, uint4* __restrict__ normal,
                                                uint4* __restrict__ albedo, size_t n) {
    int block = (int)blockIdx.x;
    if constexpr (SURF) {
        if (block < kZeroBlocks) {
            const uint4 z = make_uint4(0u, 0u, 0u, 0u);
            for (size_t i = (size_t)block * blockDim.x + threadIdx.x; i < 2 * n; i += (size_t)kZeroBlocks * blockDim.x)
                *(i < n ? normal + i : albedo + (i - n)) = z;
            return;
        }
        block -= kZeroBlocks;
    }
    const unsigned long long total = *total_p;
    const unsigned long long stride = (unsigned long long)kRasterBlocks * blockDim.x;
    const long long h = kSub / 2;
    const float sub_to_world = a.voxel / (float)kSub;
    for (unsigned long long g = (unsigned long long)block * blockDim.x + threadIdx.x; g < total; g += stride) {
        long long lo = 0, hi = n_tris - 1;
        while (lo < hi) {
            const long long mid = (lo + hi + 1) >> 1;
            if (offs[mid] <= g) lo = mid;
            else hi = mid - 1;
        }
        const TriSetup& r = setup[lo];
        const int p = (int)(g - offs[lo]);
        const long long den = r.nw * kSub;
        {
            const int pj_off = (int)((unsigned)p / (unsigned)r.w);
            const long long pi = r.i0 + (p - pj_off * r.w), pj = r.j0 + pj_off;
            const long long PX = pi * kSub + h, PY = pj * kSub + h;
            const long long ea = (r.B[0] - r.A[0]) * (PY - r.A[1]) - (r.B[1] - r.A[1]) * (PX - r.A[0]);
            const long long eb = (r.C[0] - r.B[0]) * (PY - r.B[1]) - (r.C[1] - r.B[1]) * (PX - r.B[0]);
            const long long ec = (r.A[0] - r.C[0]) * (PY - r.C[1]) - (r.A[1] - r.C[1]) * (PX - r.C[0]);
            const bool in = (ea > 0 || (ea == 0 && top_left(r.B[0] - r.A[0], r.B[1] - r.A[1]))) &&
                            (eb > 0 || (eb == 0 && top_left(r.C[0] - r.B[0], r.C[1] - r.B[1]))) &&
                            (ec > 0 || (ec == 0 && top_left(r.A[0] - r.C[0], r.A[1] - r.C[1])));
            if (!in) continue;
            const long long wnum = r.nw * r.A[2] - r.nx * (PX - r.A[0]) - r.ny * (PY - r.A[1]);
            if (wnum < 0) continue;                                  // depth below the grid
            const long long layer = floor_div_est(wnum, den);
            if (layer >= a.n) continue;
            long long v[3];
            v[r.sx] = pi;
            v[r.sy] = pj;
            v[r.sw] = layer;
            float sub[3];
            sub[r.sx] = (float)PX;
            sub[r.sy] = (float)PY;
            sub[r.sw] = (float)wnum / (float)r.nw;
            const float pos[3] = {a.origin[0] + sub[0] * sub_to_world, a.origin[1] + sub[1] * sub_to_world,
                                  a.origin[2] + sub[2] * sub_to_world};
            float lr = 0.f, lg = 0.f, lb = 0.f;
            for (int l = 0; l < a.n_lights; ++l) {
                const float dx = a.light_pos[l][0] - pos[0], dy = a.light_pos[l][1] - pos[1],
                            dz = a.light_pos[l][2] - pos[2];
                const float dist = sqrtf(dx * dx + dy * dy + dz * dz);
                const float lam = dist > 0.f ? fmaxf((dx * r.n[0] + dy * r.n[1] + dz * r.n[2]) / dist, 0.0f) : 0.0f;
                const float at = 1.0f / (a.att[l][0] + a.att[l][1] * dist + a.att[l][2] * dist * dist);
                const float kk = (a.ambient + a.diffuse * lam) * at;
                lr += kk * a.light_color[l][0];
                lg += kk * a.light_color[l][1];
                lb += kk * a.light_color[l][2];
            }
            const size_t vi = (size_t)((v[2] * a.n + v[1]) * a.n + v[0]);
            // the voxel's slot: its alpha word in base, claimed by the first fragment
            unsigned int* word = base_words + vi * 4 + 3;
            unsigned int s = __hip_atomic_load(word, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            // (a voxel is claimed once, so at most n^3 slots are taken; the
            // bound on s below only keeps a word that held anything else, were
            // base to alias another buffer, from indexing past the slots)
            const unsigned int cap = (unsigned int)a.n * a.n * a.n;
            if (s == 0u) {
                s = atomicCAS(word, 0u, kClaimed);
                if (s == 0u) {
                    const unsigned int slot = atomicAdd(counter, 1u);
                    if (slot < cap) acc[slot].voxel = (unsigned int)vi + 1u;   // read by the resolve pass only
                    s = slot + 1u;
                    atomicExch(word, s);
                }
            }
            for (int spin = 0; s == kClaimed && spin < kMaxSpin; ++spin)
                s = __hip_atomic_load(word, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            if (s == kClaimed || s > cap) continue;   // (not reached: see above; a claim is published right away)
            VoxAcc* q = acc + (s - 1u);
            atomicAdd(&q->r, to_fixed(lr * r.col[0]));
            atomicAdd(&q->g, to_fixed(lg * r.col[1]));
            atomicAdd(&q->b, to_fixed(lb * r.col[2]));
            atomicAdd(&q->count, 1u);
            if constexpr (SURF) {
                SurfAcc* u = surf + (s - 1u);
                for (int i = 0; i < 3; ++i) {
                    atomicAdd(&u->n[i], to_fixed(r.n[i]));
                    atomicAdd(&u->c[i], to_fixed(r.col[i]));
                }
            }
        }
    }
}

// One thread per used slot: write its voxel in the output grids (the other
// voxels keep the zeros of k_clear and of the raster launch's fill).
template <bool SURF>
__global__ __launch_bounds__(256) void k_resolve(const VoxAcc* __restrict__ acc, const SurfAcc* __restrict__ surf,
                                                 const unsigned int* __restrict__ counter, unsigned int cap,
                                                 float4* __restrict__ base,
                                                 float4* __restrict__ normal, float4* __restrict__ albedo) {
    const unsigned int used = min(*counter, cap);
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < used; i += (size_t)gridDim.x * blockDim.x) {
        const VoxAcc q = acc[i];
        const size_t v = (size_t)q.voxel - 1u;
        const float inv = 1.0f / ((float)q.count * kFix);
        base[v] = make_float4((float)(long long)q.r * inv, (float)(long long)q.g * inv, (float)(long long)q.b * inv,
                              1.0f);
        if constexpr (SURF) {
            const SurfAcc u = surf[i];
            normal[v] = make_float4((float)(long long)u.n[0] * inv, (float)(long long)u.n[1] * inv,
                                    (float)(long long)u.n[2] * inv, 1.0f);
            albedo[v] = make_float4((float)(long long)u.c[0] * inv, (float)(long long)u.c[1] * inv,
                                    (float)(long long)u.c[2] * inv, 1.0f);
        }
    }
}

}  // namespace

// Workspace: room for one accumulator slot per voxel (with surface attributes,
// the surface sums of every slot follow), then per-triangle setup records, the
// pixel offsets, the pixel total, the slot counter and the block sums of the
// offset scan.
size_t vct_voxelize_acc_bytes(int n, bool surface) {
    return (size_t)n * n * n * (sizeof(VoxAcc) + (surface ? sizeof(SurfAcc) : 0));
}

size_t vct_voxelize_workspace_size(int n, long long n_tris, bool surface) {
    return vct_voxelize_acc_bytes(n, surface) + (size_t)n_tris * (sizeof(TriSetup) + 8) + 256 +
           (size_t)((n_tris + kScanBlock - 1) / kScanBlock) * 8;
}

hipError_t vct_launch_voxelize(const vct_grid* g, const float* tris, const float* colors, long long n_tris,
                               const vct_voxelize_params* p, float* base, float* normal, float* albedo, void* ws,
                               hipStream_t st, EventSink& es) {
    const bool surface = normal != nullptr;
    VoxArgs a{};
    a.n = g->n;
    for (int i = 0; i < 3; ++i) a.origin[i] = g->origin[i];
    a.voxel = (float)((double)g->extent / g->n);
    a.snap_scale = (float)((double)kSub * g->n / (double)g->extent);
    a.n_lights = p->n_lights;
    for (int l = 0; l < p->n_lights; ++l)
        for (int i = 0; i < 3; ++i) {
            a.light_pos[l][i] = p->light_pos[l][i];
            a.light_color[l][i] = p->light_color[l][i];
            a.att[l][i] = p->attenuation[l][i];
        }
    a.ambient = p->ambient;
    a.diffuse = p->diffuse;
    const size_t nvox = (size_t)g->n * g->n * g->n;
    char* w = static_cast<char*>(ws);
    VoxAcc* acc = reinterpret_cast<VoxAcc*>(w);
    SurfAcc* surf = surface ? reinterpret_cast<SurfAcc*>(acc + nvox) : nullptr;
    const size_t acc_bytes = vct_voxelize_acc_bytes(g->n, surface);
    TriSetup* setup = reinterpret_cast<TriSetup*>(w + acc_bytes);
    unsigned long long* offs = reinterpret_cast<unsigned long long*>(setup + n_tris);
    unsigned long long* total = offs + n_tris;
    unsigned int* counter = reinterpret_cast<unsigned int*>(total + 1);
    unsigned long long* bsum = total + 32;      // (the 256 bytes after the offsets hold the total and the counter)
    const long long nb = (n_tris + kScanBlock - 1) / kScanBlock;
    const int fill_blocks = (int)min((nvox + 255) / 256, (size_t)16384);
    es.mark(st);
    // (with triangles, the raster pass zeroes the normal and albedo grids)
    hipLaunchKernelGGL(k_clear, dim3(fill_blocks), dim3(256), 0, st, reinterpret_cast<uint4*>(base),
                       reinterpret_cast<uint4*>(n_tris > 0 ? nullptr : normal),
                       reinterpret_cast<uint4*>(n_tris > 0 ? nullptr : albedo), nvox, counter);
    es.mark(st);
    if (n_tris > 0) {
        hipLaunchKernelGGL(k_tri_setup, dim3((unsigned)((n_tris + 255) / 256)), dim3(256), 0, st, a, tris, colors,
                           n_tris, setup, offs);
        if (n_tris <= kScanSmall) {
            hipLaunchKernelGGL(k_scan_small, dim3(1), dim3(1024), 0, st, offs, n_tris, total);
        } else {
            hipLaunchKernelGGL(k_block_sums, dim3((unsigned)nb), dim3(256), 0, st, offs, n_tris, bsum);
            hipLaunchKernelGGL(k_scan_sums, dim3(1), dim3(kScanThreads), 0, st, bsum, nb, total);
            hipLaunchKernelGGL(k_block_offsets, dim3((unsigned)nb), dim3(256), 0, st, offs, n_tris, bsum);
        }
        hipLaunchKernelGGL(k_clear_slots, dim3(1024), dim3(256), 0, st, reinterpret_cast<uint4*>(acc),
                           reinterpret_cast<uint4*>(surf), total, (unsigned long long)nvox);
        unsigned int* words = reinterpret_cast<unsigned int*>(base);
        if (surface)
            hipLaunchKernelGGL(k_raster<true>, dim3(kZeroBlocks + kRasterBlocks), dim3(256), 0, st, a, setup, offs,
                               n_tris, total, acc, surf, words, counter, reinterpret_cast<uint4*>(normal),
                               reinterpret_cast<uint4*>(albedo), nvox);
        else
            hipLaunchKernelGGL(k_raster<false>, dim3(kRasterBlocks), dim3(256), 0, st, a, setup, offs, n_tris, total,
                               acc, surf, words, counter, nullptr, nullptr, nvox);
    }
    es.mark(st);
    if (n_tris > 0) {
        if (surface)
            hipLaunchKernelGGL(k_resolve<true>, dim3(1024), dim3(256), 0, st, acc, surf, counter, (unsigned)nvox,
                               reinterpret_cast<float4*>(base), reinterpret_cast<float4*>(normal),
                               reinterpret_cast<float4*>(albedo));
        else
            hipLaunchKernelGGL(k_resolve<false>, dim3(1024), dim3(256), 0, st, acc, surf, counter, (unsigned)nvox,
                               reinterpret_cast<float4*>(base), nullptr, nullptr);
    }
    es.mark(st);
    return hipGetLastError();
}
