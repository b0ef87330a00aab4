// Mip pyramid build and level unpack (texture filtering of Section 4.3.3:
// each level is the 2x2x2 mean of the level below; mipmaps are generated after
// voxelization, Sections 4.5 and 5.4.4).
//
// One workgroup owns a B^3 block of float32 source texels (B = min(16, side)),
// stages it in LDS, writes it as the first level of the pass (when that level
// is not yet stored), and reduces it in LDS down to 1 texel, storing every
// level on the way in the pyramid's storage type.  The coarsest value of each
// block also goes to a float32 staging buffer that the next pass reads, so
// every level is computed from float32 parents and rounded exactly once.
// 256^3 needs two passes (levels 0-4, 4-8), 512^3 and 1024^3 three.
#include "texel.h"
#include "vct_internal.h"

namespace {

constexpr int kThreads = 256;
constexpr int kMaxB = 16;

struct MipPass {
    const float4* src;       // float32 logical [ns][ns][ns]
    int32_t ns;              // source side
    int32_t B;               // block side (a power of two)
    int32_t lb;              // log2(B)
    int32_t nlev;            // levels produced after the first (<= log2 B)
    int32_t first;           // pyramid level of the source
    int32_t write_first;     // store the source level too
    int32_t nblk;            // blocks a side = ns / B
    float4* stage;           // float32 output of the coarsest level of this pass (or null)
    void* pyr;
    int32_t lv_nb[VCT_MAX_LEVELS];
    uint32_t lv_off[VCT_MAX_LEVELS];
};

template <int DT>
__device__ __forceinline__ void put(const MipPass& p, int level, int x, int y, int z, float4 v) {
    // level is warp-uniform; unrolled select keeps the kernel-argument arrays in SGPRs
    int nb = 1;
    uint32_t off = 0;
#pragma unroll
    for (int l = 0; l < VCT_MAX_LEVELS; ++l)
        if (l == level) {
            nb = p.lv_nb[l];
            off = p.lv_off[l];
        }
    vct_store_texel<DT>(p.pyr, off + vct_brick_index(x, y, z, nb), v);
}

template <int DT>
__global__ __launch_bounds__(kThreads) void k_mip_block(MipPass p) {
    __shared__ float4 bufA[kMaxB * kMaxB * kMaxB];
    __shared__ float4 bufB[(kMaxB / 2) * (kMaxB / 2) * (kMaxB / 2)];
    const int B = p.B, lb = p.lb;
    const int bid = blockIdx.x;
    const int bx = bid % p.nblk;
    const int by = (bid / p.nblk) % p.nblk;
    const int bz = bid / (p.nblk * p.nblk);
    const int cnt = B * B * B;
    // all of the thread's source loads first, then the stores: issued together,
    // the loads overlap instead of each waiting behind the previous stores
    constexpr int kPer = kMaxB * kMaxB * kMaxB / kThreads;
    const float4* __restrict__ src = p.src;
    float4 v[kPer];
#pragma unroll
    for (int i = 0; i < kPer; ++i) {
        const int t = (int)threadIdx.x + i * kThreads;
        if (t < cnt) {
            const int x = t & (B - 1), y = (t >> lb) & (B - 1), z = t >> (2 * lb);
            v[i] = src[((size_t)(bz * B + z) * p.ns + (by * B + y)) * p.ns + (bx * B + x)];
        }
    }
#pragma unroll
    for (int i = 0; i < kPer; ++i) {
        const int t = (int)threadIdx.x + i * kThreads;
        if (t < cnt) {
            const int x = t & (B - 1), y = (t >> lb) & (B - 1), z = t >> (2 * lb);
            bufA[t] = v[i];
            if (p.write_first) put<DT>(p, p.first, bx * B + x, by * B + y, bz * B + z, v[i]);
        }
    }
    __syncthreads();
    float4* cur = bufA;
    float4* nxt = bufB;
    int m = B, lm = lb;
    for (int j = 1; j <= p.nlev; ++j) {
        const int pm = m;
        m >>= 1;
        --lm;
        const int c = m * m * m;
        for (int t = threadIdx.x; t < c; t += kThreads) {
            const int x = t & (m - 1), y = (t >> lm) & (m - 1), z = t >> (2 * lm);
            float4 ch[8];
#pragma unroll
            for (int q = 0; q < 8; ++q) {
                int dz = q >> 2, dy = (q >> 1) & 1, dx = q & 1;
                ch[q] = cur[((2 * z + dz) * pm + (2 * y + dy)) * pm + (2 * x + dx)];
            }
            float4 s;
            s.x = ((ch[0].x + ch[1].x) + (ch[2].x + ch[3].x)) + ((ch[4].x + ch[5].x) + (ch[6].x + ch[7].x));
            s.y = ((ch[0].y + ch[1].y) + (ch[2].y + ch[3].y)) + ((ch[4].y + ch[5].y) + (ch[6].y + ch[7].y));
            s.z = ((ch[0].z + ch[1].z) + (ch[2].z + ch[3].z)) + ((ch[4].z + ch[5].z) + (ch[6].z + ch[7].z));
            s.w = ((ch[0].w + ch[1].w) + (ch[2].w + ch[3].w)) + ((ch[4].w + ch[5].w) + (ch[6].w + ch[7].w));
            s.x *= 0.125f;
            s.y *= 0.125f;
            s.z *= 0.125f;
            s.w *= 0.125f;
            nxt[t] = s;
            int gx = bx * m + x, gy = by * m + y, gz = bz * m + z;
            put<DT>(p, p.first + j, gx, gy, gz, s);
            if (j == p.nlev && p.stage) {
                int side = p.nblk * m;
                p.stage[((size_t)gz * side + gy) * side + gx] = s;
            }
        }
        __syncthreads();
        float4* tmp = cur;
        cur = nxt;
        nxt = tmp;
    }
}

// Anisotropic levels (Section 5.1.3: mipmaps built with anisotropic
// filtering).  One thread per texel of level l >= 1, visited brick by brick,
// computes the texel for all six directions: for direction d it composites the
// two children along d's axis front to back as a ray travelling along d meets
// them (v = f + (1 - f.a) b on the four premultiplied channels) and averages
// the four pairs.  Level 1 reads the float32 base (and stores it as level 0);
// higher levels read the stored level below of the same direction.
struct AnisoPass {
    const float4* base;      // float32 logical [N][N][N] (level 1 only)
    void* pyr;
    int32_t level, side, nb, nb_child, n_base;
    uint32_t dst[6];         // texel offset of the produced level, per direction
    uint32_t src[6];         // texel offset of the level below, per direction (level 0: all 0)
};

__device__ __forceinline__ float4 over(float4 f, float4 b) {
    const float t = 1.0f - f.w;
    return make_float4(__builtin_fmaf(t, b.x, f.x), __builtin_fmaf(t, b.y, f.y), __builtin_fmaf(t, b.z, f.z),
                       __builtin_fmaf(t, b.w, f.w));
}

// Children indexed q = dz * 4 + dy * 2 + dx; axis 0 = x (bit 0), 1 = y (bit 1), 2 = z (bit 2).
__device__ __forceinline__ float4 reduce_dir(const float4 (&ch)[8], int axis, bool front_low) {
    const int bit = 1 << axis;
    float4 p[4];
    int k = 0;
#pragma unroll
    for (int q = 0; q < 8; ++q)
        if (!(q & bit)) {
            const float4 lo = ch[q], hi = ch[q | bit];
            p[k++] = front_low ? over(lo, hi) : over(hi, lo);
        }
    float4 s;
    s.x = ((p[0].x + p[1].x) + (p[2].x + p[3].x)) * 0.25f;
    s.y = ((p[0].y + p[1].y) + (p[2].y + p[3].y)) * 0.25f;
    s.z = ((p[0].z + p[1].z) + (p[2].z + p[3].z)) * 0.25f;
    s.w = ((p[0].w + p[1].w) + (p[2].w + p[3].w)) * 0.25f;
    return s;
}

template <int DT>
__global__ __launch_bounds__(256) void k_mip_aniso(AnisoPass p) {
    const uint32_t t = blockIdx.x * 256u + threadIdx.x;
    const uint32_t brick = t >> 6, w = t & 63u;
    const uint32_t nb = (uint32_t)p.nb;
    if (brick >= nb * nb * nb) return;
    const int x = (int)(brick % nb) * 4 + (int)(w & 3u), y = (int)((brick / nb) % nb) * 4 + (int)((w >> 2) & 3u),
              z = (int)(brick / (nb * nb)) * 4 + (int)(w >> 4);
    if (x >= p.side || y >= p.side || z >= p.side) return;
    const uint32_t at = vct_brick_index(x, y, z, p.nb);
    // every load before the first store: a store to the pyramid may alias the
    // later loads as far as the compiler knows, so interleaved they would run
    // one after another
    float4 ch[8], r[6];
    if (p.level == 1) {
        const float4* __restrict__ base = p.base;
#pragma unroll
        for (int q = 0; q < 8; ++q) {
            const int cx = 2 * x + (q & 1), cy = 2 * y + ((q >> 1) & 1), cz = 2 * z + (q >> 2);
            ch[q] = base[((size_t)cz * p.n_base + cy) * p.n_base + cx];
        }
    }
#pragma unroll
    for (int d = 0; d < 6; ++d) {
        if (p.level > 1) {
#pragma unroll
            for (int q = 0; q < 8; ++q)
                ch[q] = vct_load_texel<DT>(
                    p.pyr, p.src[d] + vct_brick_index(2 * x + (q & 1), 2 * y + ((q >> 1) & 1), 2 * z + (q >> 2),
                                                      p.nb_child));
        }
        r[d] = reduce_dir(ch, d >> 1, (d & 1) == 0);
    }
    if (p.level == 1) {
#pragma unroll
        for (int q = 0; q < 8; ++q)
            vct_store_texel<DT>(p.pyr,
                                vct_brick_index(2 * x + (q & 1), 2 * y + ((q >> 1) & 1), 2 * z + (q >> 2), p.nb_child),
                                ch[q]);
    }
#pragma unroll
    for (int d = 0; d < 6; ++d) vct_store_texel<DT>(p.pyr, p.dst[d] + at, r[d]);
}

template <int DT>
hipError_t run_build_aniso(const PyrLayout& L, const float* base, void* pyr, hipStream_t s, EventSink& es) {
    AnisoPass p{};
    p.base = reinterpret_cast<const float4*>(base);
    p.pyr = pyr;
    p.n_base = L.n;
    for (int l = 1; l < L.levels; ++l) {
        p.level = l;
        p.side = L.n >> l;
        p.nb = L.nb[l];
        p.nb_child = L.nb[l - 1];
        for (int d = 0; d < 6; ++d) {
            p.dst[d] = (uint32_t)L.doff[d][l];
            p.src[d] = (uint32_t)L.doff[d][l - 1];
        }
        const uint32_t threads = (uint32_t)p.nb * p.nb * p.nb * 64u;
        es.mark(s);
        hipLaunchKernelGGL(k_mip_aniso<DT>, dim3((threads + 255u) / 256u), dim3(256), 0, s, p);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    es.mark(s);
    return hipSuccess;
}

template <int DT>
__global__ __launch_bounds__(256) void k_unpack(const void* __restrict__ pyr, int nl, int nb, uint32_t off,
                                                float4* __restrict__ out) {
    const uint32_t total = (uint32_t)nl * nl * nl;
    for (uint32_t t = blockIdx.x * blockDim.x + threadIdx.x; t < total; t += gridDim.x * blockDim.x) {
        int x = t % nl, y = (t / nl) % nl, z = t / (nl * nl);
        out[t] = vct_load_texel<DT>(pyr, off + vct_brick_index(x, y, z, nb));
    }
}

template <int DT>
hipError_t run_build(const PyrLayout& L, const float* base, void* pyr, hipStream_t s, EventSink& es) {
    MipPass p{};
    p.pyr = pyr;
    for (int l = 0; l < L.levels; ++l) {
        p.lv_nb[l] = L.nb[l];
        p.lv_off[l] = (uint32_t)L.off[l];
    }
    char* pb = static_cast<char*>(pyr);
    float4* stage[2] = {reinterpret_cast<float4*>(pb + L.stage_off_bytes[0]),
                        reinterpret_cast<float4*>(pb + L.stage_off_bytes[1])};
    const float4* src = reinterpret_cast<const float4*>(base);
    int ns = L.n, first = 0, write_first = 1, si = 0;
    for (;;) {
        int B = ns < kMaxB ? ns : kMaxB;
        int lb = vct_log2i(B);
        int nlev = lb < (L.levels - 1 - first) ? lb : (L.levels - 1 - first);
        bool last = (first + nlev == L.levels - 1);
        p.src = src;
        p.ns = ns;
        p.B = B;
        p.lb = lb;
        p.nlev = nlev;
        p.first = first;
        p.write_first = write_first;
        p.nblk = ns / B;
        p.stage = last ? nullptr : stage[si];
        int nblocks = p.nblk * p.nblk * p.nblk;
        es.mark(s);
        hipLaunchKernelGGL(k_mip_block<DT>, dim3(nblocks), dim3(kThreads), 0, s, p);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
        if (last) {
            es.mark(s);
            break;
        }
        src = stage[si];
        ns >>= nlev;
        first += nlev;
        write_first = 0;
        si ^= 1;
    }
    return hipSuccess;
}

}  // namespace

hipError_t vct_launch_build_mips(const PyrLayout& L, const float* base, void* pyr, hipStream_t s, EventSink& es) {
    if (L.aniso && L.levels > 1) {   // (a single level is level 0 alone: the isotropic pack below)
        switch (L.dtype) {
            case VCT_F32: return run_build_aniso<VCT_F32>(L, base, pyr, s, es);
            case VCT_F16: return run_build_aniso<VCT_F16>(L, base, pyr, s, es);
            default: return run_build_aniso<VCT_BF16>(L, base, pyr, s, es);
        }
    }
    switch (L.dtype) {
        case VCT_F32: return run_build<VCT_F32>(L, base, pyr, s, es);
        case VCT_F16: return run_build<VCT_F16>(L, base, pyr, s, es);
        default: return run_build<VCT_BF16>(L, base, pyr, s, es);
    }
}

hipError_t vct_launch_unpack(const PyrLayout& L, const void* pyr, int level, int direction, float* out,
                             hipStream_t s) {
    int nl = L.n >> level;
    uint32_t total = (uint32_t)nl * nl * nl;
    int blocks = (int)((total + 255) / 256);
    if (blocks > 65536) blocks = 65536;
    float4* o = reinterpret_cast<float4*>(out);
    uint32_t off = (uint32_t)L.doff[direction][level];
    switch (L.dtype) {
        case VCT_F32: hipLaunchKernelGGL(k_unpack<VCT_F32>, dim3(blocks), dim3(256), 0, s, pyr, nl, L.nb[level], off, o); break;
        case VCT_F16: hipLaunchKernelGGL(k_unpack<VCT_F16>, dim3(blocks), dim3(256), 0, s, pyr, nl, L.nb[level], off, o); break;
        default: hipLaunchKernelGGL(k_unpack<VCT_BF16>, dim3(blocks), dim3(256), 0, s, pyr, nl, L.nb[level], off, o); break;
    }
    return hipGetLastError();
}
