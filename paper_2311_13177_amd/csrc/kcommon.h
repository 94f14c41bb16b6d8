// Device-side helpers shared by the HIP kernels of libvp (gfx950).
//
// Every kernel walks a list of work items (Task) with a grid-stride loop, so one
// launch can cover one slice or many slices of different sizes; each item reads its
// slice descriptor. Per-voxel and per-pixel summation orders depend only on the
// slice's own plan (bins ascending, blade parts in plan order, fixed tap order), never
// on the batch, the tile shape or the wave that happens to hold the element, so every
// tile shape gives the same bits.
//
// Uniform data (work items, descriptors, shear table, blade and knot tables) is read
// through constant-address-space pointers so that it lands in scalar registers.
#pragma once

#include <hip/hip_runtime.h>

#include "vp.h"
#include "vp_internal.h"

namespace vp {
#define AS4 __attribute__((address_space(4)))

template <class T>
__device__ __forceinline__ const AS4 T* cst(const T* p) {
    return (const AS4 T*)(const void*)p;
}

// Field of the work item's slice descriptor (descriptor array or the inline copy).
#define DF(field) (a.descs ? cst(a.descs + slice)->field : a.one.field)

// ------------------------------------------------------------------ helpers

// Floating-point contraction is off for every kernel (no fusing the compiler chooses by
// context), so a value's bits depend only on the source expression; the fused
// multiply-adds are written out.
__device__ __forceinline__ float2 cmul(float2 a, float2 b) {
    return make_float2(__builtin_fmaf(a.x, b.x, -(a.y * b.y)), __builtin_fmaf(a.x, b.y, a.y * b.x));
}
__device__ __forceinline__ float2 cadd(float2 a, float2 b) { return make_float2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ float2 csub(float2 a, float2 b) { return make_float2(a.x - b.x, a.y - b.y); }
__device__ __forceinline__ float2 cscale(float2 a, float s) { return make_float2(a.x * s, a.y * s); }
// (sign * i) * a
template <int SIGN>
__device__ __forceinline__ float2 mul_i(float2 a) {
    return SIGN > 0 ? make_float2(-a.y, a.x) : make_float2(a.y, -a.x);
}
// acc + w * a, one fused multiply-add per component
__device__ __forceinline__ float2 cfma(float w, float2 a, float2 acc) {
    return make_float2(__builtin_fmaf(w, a.x, acc.x), __builtin_fmaf(w, a.y, acc.y));
}
// SplitMix64 (Steele, Lea and Flood, 2014): the output for state x.
__device__ __forceinline__ unsigned long long splitmix64(unsigned long long x) {
    unsigned long long z = x + 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}
// Whether blade b takes part in the step with 0-based index st (operator calls, with no
// step counter, take every blade).
__device__ __forceinline__ bool active_blade(int sched, unsigned seed, const int* stepp, int st, int B, int b) {
    if (sched == VP_SCHED_ALL_BLADES || stepp == nullptr) return true;
    if (sched == VP_SCHED_CYCLIC) return b == st % B;
    const unsigned long long x = ((unsigned long long)seed << 32) | (unsigned)st;
    return (unsigned long long)b == splitmix64(x) % (unsigned long long)B;
}
__device__ __forceinline__ int read_step(const int* stepp) { return stepp ? *cst(stepp) : 0; }
// The step as the step's last kernel reads it (a.snap): the copy its first kernel took,
// while block 0 of the last kernel advances the counter itself.
__device__ __forceinline__ int read_step_at(const int* stepp, int snap) {
    return stepp ? *cst(snap ? stepp + kSnapWord : stepp) : 0;
}

// Block 0 of a step's first kernel: copy each slice's step counter to its snapshot word.
// No kernel of the step writes the counter before the last one, and only the last one
// reads the snapshot.
__device__ __forceinline__ void step_snapshot(const KArgs& a) {
    if (blockIdx.x != 0) return;
    for (int slice = threadIdx.x; slice < a.nslices; slice += blockDim.x) {
        int* const stepp = a.descs ? a.descs[slice].step : a.one.step;
        if (stepp) stepp[kSnapWord] = *stepp;
    }
}
// Block 0 of a step's last kernel: advance each slice's counter below its step limit,
// from the snapshot. Every work item of this kernel reads the snapshot, none the counter,
// so the new value is seen only by the kernels of the next step.
__device__ __forceinline__ void step_advance(const KArgs& a) {
    if (blockIdx.x != 0) return;
    for (int slice = threadIdx.x; slice < a.nslices; slice += blockDim.x) {
        int* const stepp = a.descs ? a.descs[slice].step : a.one.step;
        const int limit = a.descs ? a.descs[slice].step_limit : a.one.step_limit;
        if (stepp) {
            const int st = stepp[kSnapWord];
            if (st < limit) *stepp = st + 1;
        }
    }
}

// Charbonnier weight d / sqrt(|d|^2 + eps^2): the gradient of sqrt(|d|^2 + eps^2) - eps.
// The hardware reciprocal square root (about 1 ulp). Callers pass eps2 = max(eps^2,
// FLT_MIN) (charb_eps2), so its argument is a normal number and needs no clamp.
__device__ __forceinline__ float charb_eps2(float eps) { return fmaxf(eps * eps, 1.17549435e-38f); }
__device__ __forceinline__ float2 charb_w(float2 dlt, float eps2) {
    const float q = __builtin_fmaf(dlt.x, dlt.x, __builtin_fmaf(dlt.y, dlt.y, eps2));
    return cscale(dlt, __builtin_amdgcn_rsqf(q));
}

// Work-item index of a block. The dispatcher deals consecutive blocks to the eight XCDs
// in turn, each XCD with its own L2; renumbering gives every XCD a contiguous run of
// work items, so neighbouring items (adjacent tiles, the bin chunks and knots of one
// tile) share their halos and blade regions in one L2. A bijection on [0, grid).
// Word 3 of a raw buffer resource on this architecture, and a byte offset beyond any
// buffer used here (loads there return zero).
constexpr int kBufferFlags = 0x00020000;
constexpr int kBufferOut = 0x7ffffff0;

__device__ __forceinline__ int xcd_item(int block, int grid) {
    const int g8 = grid & ~(kXcds - 1);
    if (block >= g8) return block;
    return (block % kXcds) * (g8 / kXcds) + block / kXcds;
}

// Buffer resource over a plane of `count` complex values (count 0: an empty buffer).
__device__ __forceinline__ __amdgpu_buffer_rsrc_t plane_rsrc(const float2* base, int count) {
    return __builtin_amdgcn_make_buffer_rsrc((void*)base, (short)0, count * (int)sizeof(float2), kBufferFlags);
}
// Element `idx` of a buffer of complex values; a negative index reads zero (out of range).
__device__ __forceinline__ float2 buffer_c64(__amdgpu_buffer_rsrc_t r, int idx) {
    const int byte = idx >= 0 ? idx * (int)sizeof(float2) : kBufferOut;
    return __builtin_bit_cast(float2, __builtin_amdgcn_raw_buffer_load_b64(r, byte, 0, 0));
}

// ------------------------------------------------------------------ LDS staging
//
// A rectangular region (rows x cols) of an n x n image, origin (gy0, gx0), is staged
// into LDS with zeros outside the image by the NT threads of a work item. Each thread
// owns region elements threadIdx.x + k * NT (k < SE); their image offsets are computed once per work
// item, and the next plane's values are loaded into registers while the current plane
// is being consumed (double-buffered LDS, one barrier per plane).

// P planes (images of the same size, same region) are staged per phase; plane p of a
// phase occupies buf[p * re, (p + 1) * re). A null plane pointer stages zeros.
// Whole-wave lane shifts by one (DPP wave_shr / wave_shl): lane i receives lane i - 1
// (shfl_up1) or lane i + 1 (shfl_down1); the lane without a source reads zero.
template <int CTRL>
__device__ __forceinline__ float dpp_f(float v) {
    return __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v), CTRL, 0xf, 0xf, true));
}
__device__ __forceinline__ float2 shfl_up1(float2 v) { return make_float2(dpp_f<0x138>(v.x), dpp_f<0x138>(v.y)); }
__device__ __forceinline__ float2 shfl_down1(float2 v) { return make_float2(dpp_f<0x130>(v.x), dpp_f<0x130>(v.y)); }
// Lane l's value of v, for the whole wave (v_readlane: a wave-uniform value in SGPRs, no
// memory access).
__device__ __forceinline__ float2 lane_f2(float2 v, int l) {
    return make_float2(__builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, v.x), l)),
                       __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, v.y), l)));
}

template <int SE, int P, int NT = kThreads>
struct Stager {
    int off[SE];
    int re;
    __device__ void init(int rows, int cols, int gy0, int gx0, int n) {
        re = rows * cols;
#pragma unroll
        for (int k = 0; k < SE; ++k) {
            const int i = threadIdx.x + k * NT;
            int o = -1;
            if (i < re) {
                const int r = i / cols, c = i - (i / cols) * cols;
                const int gy = gy0 + r, gx = gx0 + c;
                if (gy >= 0 && gy < n && gx >= 0 && gx < n) o = gy * n + gx;
            }
            off[k] = i < re ? o : -2;
        }
    }
    // Buffer loads with the plane as the buffer: an element outside the image (or a null
    // plane, whose buffer is empty) is out of range and reads as zero without a branch
    // or a memory access.
    __device__ void fetch(const float2* const (&img)[P], int nn, float2 (&pre)[P][SE]) const {
#pragma unroll
        for (int p = 0; p < P; ++p) {
            const __amdgpu_buffer_rsrc_t r = plane_rsrc(img[p], img[p] ? nn : 0);
#pragma unroll
            for (int k = 0; k < SE; ++k) pre[p][k] = buffer_c64(r, off[k]);
        }
    }
    __device__ void store(float2* buf, const float2 (&pre)[P][SE]) const {
#pragma unroll
        for (int p = 0; p < P; ++p)
#pragma unroll
            for (int k = 0; k < SE; ++k)
                if (off[k] != -2) buf[p * re + threadIdx.x + k * NT] = pre[p][k];
    }
};

}  // namespace vp
