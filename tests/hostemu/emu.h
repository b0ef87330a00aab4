// Host emulation of the gfx950 execution model for the library's kernels
// (test infrastructure: the checked CPU build).  Force-included before every
// library source, which is then compiled as plain C++ for the host:
//   * a workgroup runs as cooperative fibers, one per work item, grouped in
//     64-lane waves; __syncthreads is a barrier over the workgroup's live
//     fibers, and cross-lane operations (ballot, readlane, shuffles, DPP row
//     and quad permutes, permlane swaps) are barriers over the wave that
//     exchange the lanes' values, so the reduction butterflies run exactly as
//     written;
//   * a cross-lane operation reached by lanes at different call sites, a read
//     from a lane that has exited, or a deadlock is reported as an error;
//   * buffer-resource loads (raw, structured, scalar) follow the hardware's
//     range rule (bytes past the resource's range read as zero) and are also
//     checked against the allocations the harness registered, so a resource
//     wider than its memory is an error rather than a silent read;
//   * texel and accumulator indices go through the VCT_CHECK_TEXEL and
//     VCT_CHECK_ACC hooks, checked against the current call's bounds.
// Work-group shared variables become function statics (shared by the fibers
// of a workgroup; workgroups run one after another).
#pragma once

#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <algorithm>
#include <type_traits>

// device-side overloads the kernels call unqualified
using std::isfinite;
using std::max;
using std::min;

#undef __shared__
#define __shared__ static
#ifndef __align__
#define __align__(x) __attribute__((aligned(x)))
#endif
#ifndef HIP_SYMBOL
#define HIP_SYMBOL(x) x
#endif
#define __launch_bounds__(...)

struct EmuDim {
    unsigned x, y, z;
};

void emu_fail(const char* fmt, ...) __attribute__((noreturn, format(printf, 1, 2)));

// ---- work items
EmuDim emu_thread_idx();
extern EmuDim emu_block_idx, emu_block_dim, emu_grid_dim;
#define threadIdx (emu_thread_idx())
#define blockIdx (emu_block_idx)
#define blockDim (emu_block_dim)
#define gridDim (emu_grid_dim)

void emu_syncthreads(const char* site);
#define EMU_SITE2(f, l) f ":" #l
#define EMU_SITE1(f, l) EMU_SITE2(f, l)
#define EMU_SITE EMU_SITE1(__FILE__, __LINE__)
#define __syncthreads() emu_syncthreads(EMU_SITE)

// ---- cross-lane operations (64-lane waves)
enum EmuOp { EMU_BALLOT, EMU_READLANE, EMU_SHFL_XOR, EMU_DPP, EMU_PL16, EMU_PL32 };
struct EmuPair {
    uint32_t v[2];
    uint32_t operator[](int i) const { return v[i]; }
};
uint64_t emu_wave_op(EmuOp op, const char* site, uint64_t a, uint64_t b, int param);

#define __ballot(p) emu_wave_op(EMU_BALLOT, EMU_SITE, (p) ? 1u : 0u, 0, 0)
#define __builtin_amdgcn_readlane(v, l) ((int)emu_wave_op(EMU_READLANE, EMU_SITE, (uint32_t)(v), 0, (l)))
// (every readfirstlane in the kernels reads a wave-uniform value or takes the
// lane's own view of a footprint test: its own value)
#define __builtin_amdgcn_readfirstlane(v) (v)
// the wave-uniform footprint test, from each lane's own view: it always shares
// its own footprint, so the scalar-load path runs for every lane
#define VCT_WAVE_AGREES(differs) (!(differs))

template <typename T>
inline T emu_shfl_xor(T v, int mask, int width = 64) {
    static_assert(sizeof(T) == 4 || sizeof(T) == 8, "32- or 64-bit values only");
    if (width != 64) emu_fail("shuffle width %d", width);
    uint64_t u = 0;
    memcpy(&u, &v, sizeof(T));
    const uint64_t r = emu_wave_op(EMU_SHFL_XOR, "shfl_xor", u, 0, mask);
    T out;
    memcpy(&out, &r, sizeof(T));
    return out;
}
#define __shfl_xor emu_shfl_xor
#define __builtin_amdgcn_mov_dpp(v, ctrl, rm, bm, bc) ((int)emu_wave_op(EMU_DPP, "dpp", (uint32_t)(v), 0, (ctrl)))
inline EmuPair emu_permlane_swap(EmuOp op, uint32_t a, uint32_t b) {
    const uint64_t r = emu_wave_op(op, "permlane_swap", a, b, 0);
    return EmuPair{{(uint32_t)r, (uint32_t)(r >> 32)}};
}
#define __builtin_amdgcn_permlane16_swap(a, b, fi, bc) emu_permlane_swap(EMU_PL16, (a), (b))
#define __builtin_amdgcn_permlane32_swap(a, b, fi, bc) emu_permlane_swap(EMU_PL32, (a), (b))

// ---- arithmetic builtins
inline float emu_fmed3f(float a, float b, float c) { return fmaxf(fminf(a, b), fminf(fmaxf(a, b), c)); }
#define __builtin_amdgcn_fmed3f(a, b, c) emu_fmed3f((a), (b), (c))
#define __builtin_amdgcn_logf(x) log2f(x)
#define __builtin_amdgcn_rcpf(x) (1.0f / (x))
#define __builtin_amdgcn_sched_barrier(x) ((void)0)
#define __popcll(x) __builtin_popcountll(x)

inline float __int_as_float(int v) { float f; memcpy(&f, &v, 4); return f; }
inline float __uint_as_float(unsigned v) { float f; memcpy(&f, &v, 4); return f; }
inline int __float_as_int(float f) { int v; memcpy(&v, &f, 4); return v; }
inline unsigned __float_as_uint(float f) { unsigned v; memcpy(&v, &f, 4); return v; }

// ---- atomics (fibers run on one host thread: plain read-modify-writes)
template <typename T>
inline T atomicAdd(T* p, T v) {
    const T old = *p;
    *p = old + v;
    return old;
}
template <typename T>
inline T atomicCAS(T* p, T cmp, T v) {
    const T old = *p;
    if (old == cmp) *p = v;
    return old;
}
template <typename T>
inline T atomicExch(T* p, T v) {
    const T old = *p;
    *p = v;
    return old;
}
#ifndef __HIP_MEMORY_SCOPE_AGENT
#define __HIP_MEMORY_SCOPE_AGENT 3
#endif
#define __hip_atomic_load(p, order, scope) (*(p))

// ---- memory checks
void emu_check_texel(uint64_t idx, const char* site);
void emu_check_acc(uint64_t idx, const char* site);
#define VCT_CHECK_TEXEL(idx) emu_check_texel((uint64_t)(idx), EMU_SITE)
#define VCT_CHECK_ACC(idx) emu_check_acc((uint64_t)(idx), EMU_SITE)

// ---- launches
void emu_run_grid(dim3 grid, dim3 block, void (*body)(void*), void* ctx);
template <typename F, typename... A>
inline void emu_launch(F f, dim3 grid, dim3 block, A... args) {
    auto call = [&]() { f(args...); };
    emu_run_grid(grid, block, [](void* c) { (*static_cast<decltype(call)*>(c))(); }, &call);
}
#define hipLaunchKernelGGL(kernel, grid, block, shmem, stream, ...) emu_launch((kernel), dim3(grid), dim3(block), __VA_ARGS__)
