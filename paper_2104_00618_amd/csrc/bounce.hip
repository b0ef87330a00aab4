// A further light bounce inside the voxel grid (Section 6.2.2 "Algorithm
// Limitations": more bounces need a texture of average surface normals and
// cones traced again from the voxels hit; Sections 6.2.4 and 5.1.3: indirect
// light inserted into a further 3D texture, as deferred voxel cone tracing
// does).  From every surface voxel (alpha > 0, average normal of length >=
// 1/100) the diffuse cones of the cone set march through the given pyramid,
// about the voxel's unit average normal, from the voxel centre offset by
// normal_offset voxels; the voxel becomes
//   out.rgb = base.rgb + base.a * albedo.rgb * sum_q w_q C_q,  out.a = base.a,
// and every other voxel keeps its base value.
//
// Launch.  Surface voxels are sparse (a few percent of the grid), so they are
// first compacted into a list and the march runs over full waves of them:
//   k_flag   one 16^3 block of voxels per workgroup (blocks in Morton order,
//            rows of 16 voxels inside, so a wave reads 256-byte runs): the
//            alpha test is a ballot per 64 voxels, stored as a 64-bit mask,
//            plus the block's count; copies base into out on the way unless
//            out is base;
//   k_scan   exclusive scan of the block counts (one workgroup) and the total;
//   k_list   writes the linear index of every flagged voxel at its offset, so
//            consecutive entries are neighbours in space (neighbouring lanes
//            march similar cones);
//   k_gather a fixed grid of workgroups takes tiles of 64 list entries (the
//            length is known on the device only) from a counter per XCD over
//            that XCD's contiguous run; one wave per cone of the tile's voxels.
#include "march.h"

namespace {

using namespace vct;

constexpr uint32_t kBlockVox = 4096;      // voxels per compaction workgroup (one 16^3 block)
constexpr int kScanThreads = 1024;
constexpr float kMinNormal2 = 1e-4f;      // (1/100)^2: shorter average normals have no direction
constexpr int kGatherBlocks = 2048;       // multiple of 8 (XCDs); workgroups beyond residency find no tile

// Bits 0, 3, 6, ... of v packed into bits 0, 1, 2, ... (inverse of a 3-way bit interleave, 10 bits out).
__device__ __forceinline__ uint32_t compact3(uint32_t v) {
    v &= 0x09249249u;
    v = (v ^ (v >> 2)) & 0x030c30c3u;
    v = (v ^ (v >> 4)) & 0x0300f00fu;
    v = (v ^ (v >> 8)) & 0xff0000ffu;
    v = (v ^ (v >> 16)) & 0x000003ffu;
    return v;
}

// Linear index (z * N + y) * N + x of visit index m, N = 2^lg: blocks of
// s^3 voxels (s = min(N, 16)) in Morton order of the block coordinates (x in
// bit 0, y in bit 1, z in bit 2), voxels inside a block row by row (x fastest).
__device__ __forceinline__ uint32_t visit_to_linear(uint32_t m, int lg) {
    const int sl = lg < 4 ? lg : 4;
    const uint32_t l = m & ((1u << (3 * sl)) - 1u), blk = m >> (3 * sl);
    const uint32_t sm = (1u << sl) - 1u;
    const uint32_t x = (compact3(blk) << sl) | (l & sm);
    const uint32_t y = (compact3(blk >> 1) << sl) | ((l >> sl) & sm);
    const uint32_t z = (compact3(blk >> 2) << sl) | (l >> (2 * sl));
    return (z << (2 * lg)) | (y << lg) | x;
}

__global__ __launch_bounds__(256) void k_flag(const float4* __restrict__ base, float4* __restrict__ copy,
                                              unsigned long long* __restrict__ masks, uint32_t* __restrict__ counts,
                                              uint32_t nvox, int lg) {
    constexpr int kIter = kBlockVox / 4 / 64;    // 64-voxel groups per wave
    __shared__ uint32_t s_cnt[4];
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const uint32_t w0 = blockIdx.x * kBlockVox + wave * (kBlockVox / 4);
    // all loads first, so that a wave has its 16 groups in flight at once
    float4 val[kIter];
    uint32_t vid[kIter];
#pragma unroll
    for (int i = 0; i < kIter; ++i) {
        const uint32_t m = w0 + i * 64 + lane;
        vid[i] = m < nvox ? visit_to_linear(m, lg) : 0u;
        val[i] = m < nvox ? base[vid[i]] : make_float4(0.f, 0.f, 0.f, 0.f);
    }
    uint32_t cnt = 0;
#pragma unroll
    for (int i = 0; i < kIter; ++i) {
        const uint32_t first = w0 + i * 64;
        const bool in = first + lane < nvox;
        if (copy && in) copy[vid[i]] = val[i];
        const unsigned long long bal = __ballot(in && val[i].w > 0.0f);
        if (lane == 0 && first < nvox) masks[first >> 6] = bal;
        cnt += (uint32_t)__popcll(bal);
    }
    if (lane == 0) s_cnt[wave] = cnt;
    __syncthreads();
    if (threadIdx.x == 0) counts[blockIdx.x] = s_cnt[0] + s_cnt[1] + s_cnt[2] + s_cnt[3];
}

// In place: counts[i] becomes the sum of counts[0..i); *total the sum of all.
// Also resets the gather's per-XCD tile counters (each on a cache line of its
// own: the XCDs would otherwise serialise on one line).
__global__ __launch_bounds__(kScanThreads) void k_scan(uint32_t* __restrict__ counts, uint32_t n,
                                                       uint32_t* __restrict__ total, uint32_t* __restrict__ queue) {
    if (threadIdx.x < 8) queue[threadIdx.x * 64] = 0u;
    __shared__ uint32_t s[kScanThreads];
    const uint32_t per = (n + kScanThreads - 1) / kScanThreads;
    const uint32_t b = threadIdx.x * per, e = min(b + per, n);
    uint32_t own = 0;
    for (uint32_t i = b; i < e; ++i) own += counts[i];
    s[threadIdx.x] = own;
    __syncthreads();
    for (int off = 1; off < kScanThreads; off <<= 1) {   // inclusive Hillis-Steele scan
        const uint32_t add = threadIdx.x >= (unsigned)off ? s[threadIdx.x - off] : 0u;
        __syncthreads();
        s[threadIdx.x] += add;
        __syncthreads();
    }
    uint32_t run = s[threadIdx.x] - own;
    for (uint32_t i = b; i < e; ++i) {
        const uint32_t c = counts[i];
        counts[i] = run;
        run += c;
    }
    if (threadIdx.x == kScanThreads - 1) *total = s[kScanThreads - 1];
}

__global__ __launch_bounds__(256) void k_list(const unsigned long long* __restrict__ masks,
                                              const uint32_t* __restrict__ offs, uint32_t nvox, int lg,
                                              uint32_t* __restrict__ list) {
    __shared__ uint32_t s_cnt[4];
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const uint32_t w0 = blockIdx.x * kBlockVox + wave * (kBlockVox / 4);
    uint32_t cnt = 0;
    for (uint32_t i = 0; i < kBlockVox / 4 && w0 + i < nvox; i += 64) cnt += (uint32_t)__popcll(masks[(w0 + i) >> 6]);
    if (lane == 0) s_cnt[wave] = cnt;
    __syncthreads();
    uint32_t pos = offs[blockIdx.x];
    for (int w = 0; w < wave; ++w) pos += s_cnt[w];
    const unsigned long long below = (1ull << lane) - 1ull;
    for (uint32_t i = 0; i < kBlockVox / 4 && w0 + i < nvox; i += 64) {
        const unsigned long long mk = masks[(w0 + i) >> 6];
        const uint32_t at = pos + (uint32_t)__popcll(mk & below);   // (< nvox: one bit per voxel)
        if (((mk >> lane) & 1ull) && at < nvox) list[at] = visit_to_linear(w0 + i + lane, lg);
        pos += (uint32_t)__popcll(mk);
    }
}

struct BounceArgs {
    const float4* base;
    const float4* normal;
    const float4* albedo;
    float4* out;
    const uint32_t* list;
    const uint32_t* total;
    uint32_t* queue;          // 8 tile counters, one per XCD, 64 words apart
    int32_t lg;
};

// Workgroup = 64 listed voxels x u cones: wave q marches cone q of the 64
// voxels (neighbours in space with, mostly, one normal, so the lanes of a wave
// march nearly the same cone); the weighted colours meet in LDS and wave 0
// sums them in cone order (the order of the forward trace's diffuse sum).
// Tiles of 64 list entries are taken from the XCD's own contiguous run through
// an atomic counter, so faster workgroups take more tiles.
template <int DT, bool ANISO>
__global__ __launch_bounds__(1024) void k_gather(TraceArgs a, BounceArgs b) {
    __shared__ LevelTable T;
    __shared__ DirSlot<ANISO> D;
    __shared__ float s_c[VCT_MAX_DIFFUSE][3][64];
    __shared__ uint32_t s_tile;
    load_level_table(a, &T);
    load_dir_table(a, &D);
    const uint32_t total = min(*b.total, 1u << (3 * b.lg));   // (the list holds at most n^3 entries)
    const uint32_t nt = (total + 63u) / 64u;
    const uint32_t per_xcd = (nt + 7u) / 8u;
    const uint32_t xcd = blockIdx.x & 7u;
    const uint32_t begin = xcd * per_xcd, end = min(begin + per_xcd, nt);
    const int q = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const uint32_t mask = (1u << b.lg) - 1u;
    for (;;) {
        __syncthreads();                                     // level table loaded; last tile's sums consumed
        if (threadIdx.x == 0) s_tile = begin + atomicAdd(&b.queue[xcd * 64], 1u);
        __syncthreads();
        const uint32_t tile = s_tile;
        if (tile >= end) break;                              // workgroup-uniform
        const uint32_t i = tile * 64u + lane;
        uint32_t v = 0;
        bool live = false;
        float r = 0.f, g = 0.f, bl = 0.f;
        if (i < total) {
            v = b.list[i];
            const float4 nr = b.normal[v];
            live = nr.x * nr.x + nr.y * nr.y + nr.z * nr.z >= kMinNormal2;
            if (live) {
                PixelSetup P;
                set_frame(P, nr);
                // the voxel centre (i + 1/2 in texel units) is exact in float
                const float x = (float)(v & mask), y = (float)((v >> b.lg) & mask), z = (float)(v >> (2 * b.lg));
                set_origin(a, P, df{x + 0.5f, 0.0f}, df{y + 0.5f, 0.0f}, df{z + 0.5f, 0.0f});
                const Cone c = cone_for_slot(a, P, q, make_float3(0.f, 0.f, 0.f));   // diffuse: no camera
                const MarchResult m = march<DT, ANISO, kShareFootprint<DT>>(a, T, c, dir_ptr(D));
                r = m.r;
                g = m.g;
                bl = m.b;
            }
        }
        s_c[q][0][lane] = r;
        s_c[q][1][lane] = g;
        s_c[q][2][lane] = bl;
        __syncthreads();
        if (q == 0 && live) {
            float sr = 0.f, sg = 0.f, sb = 0.f;
            for (int k = 0; k < a.n_diffuse; ++k) {
                const float wk = a.weight[k];
                sr = __builtin_fmaf(wk, s_c[k][0][lane], sr);
                sg = __builtin_fmaf(wk, s_c[k][1][lane], sg);
                sb = __builtin_fmaf(wk, s_c[k][2][lane], sb);
            }
            const float4 s = b.base[v];
            const float4 al = b.albedo[v];
            b.out[v] = make_float4(__builtin_fmaf(s.w * al.x, sr, s.x), __builtin_fmaf(s.w * al.y, sg, s.y),
                                   __builtin_fmaf(s.w * al.z, sb, s.z), s.w);
        }
    }
}

template <int DT>
void launch_gather(const TraceArgs& a, const BounceArgs& b, hipStream_t st) {
    if (a.aniso)
        hipLaunchKernelGGL((k_gather<DT, true>), dim3(kGatherBlocks), dim3(64 * a.n_diffuse), 0, st, a, b);
    else
        hipLaunchKernelGGL((k_gather<DT, false>), dim3(kGatherBlocks), dim3(64 * a.n_diffuse), 0, st, a, b);
}

size_t align256(size_t v) { return (v + 255) & ~size_t(255); }

struct BounceWs {
    size_t masks, counts, total, queue, list, bytes;
};

BounceWs bounce_ws(int n) {
    const size_t nvox = (size_t)n * n * n;
    const size_t nblk = (nvox + kBlockVox - 1) / kBlockVox;
    BounceWs w{};
    w.masks = 0;
    w.counts = align256(((nvox + 63) / 64) * 8);
    w.total = w.counts + align256(nblk * 4);
    w.queue = w.total + 256;                     // 8 counters, 256 bytes apart (one cache line each)
    w.list = w.queue + 2048;
    w.bytes = w.list + align256(nvox * 4);
    return w;
}

}  // namespace

size_t vct_bounce_workspace_size(int n) { return bounce_ws(n).bytes; }

hipError_t vct_launch_bounce(const TraceArgs& a, int dtype, const float* base, const float* normal,
                             const float* albedo, float* out, void* ws, hipStream_t st, EventSink& es) {
    const int n = a.n;
    int lg = 0;
    while ((1 << lg) < n) ++lg;
    const uint32_t nvox = (uint32_t)n * n * n;
    const uint32_t nblk = (nvox + kBlockVox - 1) / kBlockVox;
    const BounceWs w = bounce_ws(n);
    char* p = static_cast<char*>(ws);
    auto* masks = reinterpret_cast<unsigned long long*>(p + w.masks);
    auto* counts = reinterpret_cast<uint32_t*>(p + w.counts);
    auto* total = reinterpret_cast<uint32_t*>(p + w.total);
    auto* queue = reinterpret_cast<uint32_t*>(p + w.queue);
    auto* list = reinterpret_cast<uint32_t*>(p + w.list);
    float4* copy = out == base ? nullptr : reinterpret_cast<float4*>(out);
    es.mark(st);
    hipLaunchKernelGGL(k_flag, dim3(nblk), dim3(256), 0, st, reinterpret_cast<const float4*>(base), copy, masks,
                       counts, nvox, lg);
    es.mark(st);
    hipLaunchKernelGGL(k_scan, dim3(1), dim3(kScanThreads), 0, st, counts, nblk, total, queue);
    es.mark(st);
    hipLaunchKernelGGL(k_list, dim3(nblk), dim3(256), 0, st, masks, counts, nvox, lg, list);
    BounceArgs b{reinterpret_cast<const float4*>(base), reinterpret_cast<const float4*>(normal),
                 reinterpret_cast<const float4*>(albedo), reinterpret_cast<float4*>(out), list, total, queue, lg};
    es.mark(st);
    if (a.n_diffuse > 0) {
        (void)vct_dispatch_dt(dtype, a.wide != 0, [&](auto dt) {   // (launch errors: hipGetLastError below)
            launch_gather<decltype(dt)::value>(a, b, st);
            return hipSuccess;
        });
    }
    es.mark(st);
    return hipGetLastError();
}
