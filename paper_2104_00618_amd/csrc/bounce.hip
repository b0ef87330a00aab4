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
//   k_flag   one 16^3 block of voxels per workgroup, visited in Morton order
//            (a wave's 64 voxels are one 4^3 brick): the alpha test is a
//            ballot, stored as one 64-bit mask per brick, plus the block's
//            count; copies base into out on the way unless out is base;
//   k_scan   exclusive scan of the block counts (one workgroup) and the total;
//   k_list   writes the linear index of every flagged voxel at its offset, so
//            the list is in Morton order and consecutive entries are
//            neighbours in space (neighbouring lanes march similar cones);
//   k_gather a fixed grid of workgroups walks the list tile by tile (the
//            length is known on the device only), each XCD taking one
//            contiguous run of tiles, one lane per surface voxel.
#include "march.h"

namespace {

using namespace vct;

constexpr uint32_t kBlockVox = 4096;      // voxels per compaction workgroup (a 16^3 Morton block)
constexpr int kScanThreads = 1024;
constexpr float kMinNormal2 = 1e-4f;      // (1/100)^2: shorter average normals have no direction
constexpr int kGatherBlocks = 2048;       // multiple of 8 (XCDs)

// Bits 0, 3, 6, ... of v packed into bits 0, 1, 2, ... (inverse of a 3-way bit interleave, 10 bits out).
__device__ __forceinline__ uint32_t compact3(uint32_t v) {
    v &= 0x09249249u;
    v = (v ^ (v >> 2)) & 0x030c30c3u;
    v = (v ^ (v >> 4)) & 0x0300f00fu;
    v = (v ^ (v >> 8)) & 0xff0000ffu;
    v = (v ^ (v >> 16)) & 0x000003ffu;
    return v;
}

// Linear index (z * N + y) * N + x of Morton index m (x in bit 0, y in bit 1, z in bit 2), N = 2^lg.
__device__ __forceinline__ uint32_t morton_to_linear(uint32_t m, int lg) {
    return (compact3(m >> 2) << (2 * lg)) | (compact3(m >> 1) << lg) | compact3(m);
}

__global__ __launch_bounds__(256) void k_flag(const float4* __restrict__ base, float4* __restrict__ copy,
                                              unsigned long long* __restrict__ masks, uint32_t* __restrict__ counts,
                                              uint32_t nvox, int lg) {
    __shared__ uint32_t s_cnt[4];
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const uint32_t w0 = blockIdx.x * kBlockVox + wave * (kBlockVox / 4);
    uint32_t cnt = 0;
    for (uint32_t i = 0; i < kBlockVox / 4; i += 64) {
        const uint32_t first = w0 + i;
        if (first >= nvox) break;                    // wave-uniform
        const uint32_t m = first + lane;
        bool f = false;
        if (m < nvox) {
            const uint32_t v = morton_to_linear(m, lg);
            const float4 b = base[v];
            if (copy) copy[v] = b;
            f = b.w > 0.0f;
        }
        const unsigned long long bal = __ballot(f);
        if (lane == 0) masks[first >> 6] = bal;
        cnt += (uint32_t)__popcll(bal);
    }
    if (lane == 0) s_cnt[wave] = cnt;
    __syncthreads();
    if (threadIdx.x == 0) counts[blockIdx.x] = s_cnt[0] + s_cnt[1] + s_cnt[2] + s_cnt[3];
}

// In place: counts[i] becomes the sum of counts[0..i); *total the sum of all.
__global__ __launch_bounds__(kScanThreads) void k_scan(uint32_t* __restrict__ counts, uint32_t n,
                                                       uint32_t* __restrict__ total) {
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
        if ((mk >> lane) & 1ull) list[pos + (uint32_t)__popcll(mk & below)] = morton_to_linear(w0 + i + lane, lg);
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
    int32_t lg;
};

template <int DT>
__device__ __forceinline__ void gather_voxel(const TraceArgs& a, const LevelTable& T, const BounceArgs& b,
                                             uint32_t v) {
    const float4 nr = b.normal[v];
    if (!(nr.x * nr.x + nr.y * nr.y + nr.z * nr.z >= kMinNormal2)) return;
    const uint32_t mask = (1u << b.lg) - 1u;
    const float x = (float)(v & mask), y = (float)((v >> b.lg) & mask), z = (float)(v >> (2 * b.lg));
    PixelSetup P;
    set_frame(P, nr);
    // the voxel centre (i + 1/2 in texel units) is exact in float
    set_origin(a, P, df{x + 0.5f, 0.0f}, df{y + 0.5f, 0.0f}, df{z + 0.5f, 0.0f});
    const float3 unused = make_float3(0.f, 0.f, 0.f);   // camera: no specular cone here
    float r = 0.f, g = 0.f, bl = 0.f;
    for (int q = 0; q < a.n_diffuse; ++q) {
        const Cone c = cone_for_slot(a, P, q, unused);
        const MarchResult m = march<DT>(a, T, c);
        const float wq = a.weight[q];
        r = __builtin_fmaf(wq, m.r, r);
        g = __builtin_fmaf(wq, m.g, g);
        bl = __builtin_fmaf(wq, m.b, bl);
    }
    const float4 s = b.base[v];
    const float4 al = b.albedo[v];
    b.out[v] = make_float4(__builtin_fmaf(s.w * al.x, r, s.x), __builtin_fmaf(s.w * al.y, g, s.y),
                           __builtin_fmaf(s.w * al.z, bl, s.z), s.w);
}

template <int DT>
__global__ __launch_bounds__(256) void k_gather(TraceArgs a, BounceArgs b) {
    __shared__ LevelTable T;
    load_level_table(a, &T);
    __syncthreads();
    const uint32_t total = *b.total;
    const uint32_t nt = (total + 255u) / 256u;
    const uint32_t per_xcd = (nt + 7u) / 8u;
    const uint32_t xcd = blockIdx.x & 7u, slot = blockIdx.x >> 3, nslot = gridDim.x >> 3;
    const uint32_t end = min((xcd + 1u) * per_xcd, nt);
    for (uint32_t tile = xcd * per_xcd + slot; tile < end; tile += nslot) {
        const uint32_t i = tile * 256u + threadIdx.x;
        if (i < total) gather_voxel<DT>(a, T, b, b.list[i]);
    }
}

template <int DT>
void launch_gather(const TraceArgs& a, const BounceArgs& b, hipStream_t st) {
    hipLaunchKernelGGL(k_gather<DT>, dim3(kGatherBlocks), dim3(256), 0, st, a, b);
}

size_t align256(size_t v) { return (v + 255) & ~size_t(255); }

struct BounceWs {
    size_t masks, counts, total, list, bytes;
};

BounceWs bounce_ws(int n) {
    const size_t nvox = (size_t)n * n * n;
    const size_t nblk = (nvox + kBlockVox - 1) / kBlockVox;
    BounceWs w{};
    w.masks = 0;
    w.counts = align256(((nvox + 63) / 64) * 8);
    w.total = w.counts + align256(nblk * 4);
    w.list = w.total + 256;
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
    auto* list = reinterpret_cast<uint32_t*>(p + w.list);
    float4* copy = out == base ? nullptr : reinterpret_cast<float4*>(out);
    es.mark(st);
    hipLaunchKernelGGL(k_flag, dim3(nblk), dim3(256), 0, st, reinterpret_cast<const float4*>(base), copy, masks,
                       counts, nvox, lg);
    es.mark(st);
    hipLaunchKernelGGL(k_scan, dim3(1), dim3(kScanThreads), 0, st, counts, nblk, total);
    es.mark(st);
    hipLaunchKernelGGL(k_list, dim3(nblk), dim3(256), 0, st, masks, counts, nvox, lg, list);
    BounceArgs b{reinterpret_cast<const float4*>(base), reinterpret_cast<const float4*>(normal),
                 reinterpret_cast<const float4*>(albedo), reinterpret_cast<float4*>(out), list, total, lg};
    es.mark(st);
    if (a.n_diffuse > 0) {
        switch (dtype) {
            case VCT_F32: launch_gather<VCT_F32>(a, b, st); break;
            case VCT_F16: launch_gather<VCT_F16>(a, b, st); break;
            default: launch_gather<VCT_BF16>(a, b, st); break;
        }
    }
    es.mark(st);
    return hipGetLastError();
}
