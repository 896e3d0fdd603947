// device_common.hpp -- gfx950 device helpers shared by the stencil kernels:
// storage <-> compute conversions, whole-wave DPP lane shifts, compile-time
// loops, and the XCD-aware workgroup remap.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>
#include <type_traits>
#include <utility>

namespace stn {

// ---------------------------------------------------------------------------
// Storage types.  bf16 is kept as its raw 16 bits; fp16 uses _Float16.
struct bf16_t {
    uint16_t bits;
};

template <typename S> struct ComputeOf { using type = float; };
template <> struct ComputeOf<double> { using type = double; };

__device__ __forceinline__ float to_compute(float v) { return v; }
__device__ __forceinline__ double to_compute(double v) { return v; }
__device__ __forceinline__ float to_compute(_Float16 v) { return (float)v; }
__device__ __forceinline__ float to_compute(bf16_t v) {
    return __uint_as_float(((uint32_t)v.bits) << 16);
}

template <typename S> __device__ __forceinline__ S from_compute(float v);
template <typename S> __device__ __forceinline__ S from_compute(double v);
template <> __device__ __forceinline__ float from_compute<float>(float v) { return v; }
template <> __device__ __forceinline__ double from_compute<double>(double v) { return v; }
template <> __device__ __forceinline__ _Float16 from_compute<_Float16>(float v) {
    // The empty asm makes the FP32 value opaque, so the compiler cannot fuse the
    // FMA that produced it with this conversion (v_fma_mixlo_f16 rounds the exact
    // a*b+c straight to FP16): every result is rounded to FP32 first, then to
    // FP16, wherever the kernel stores it.
    asm("" : "+v"(v));
    return (_Float16)v;  // v_cvt_f16_f32, round to nearest even
}
template <> __device__ __forceinline__ bf16_t from_compute<bf16_t>(float v) {
    // round to nearest even (gfx950 converts in one instruction,
    // v_cvt_pk_bf16_f32); a NaN stays a NaN
    bf16_t r;
    r.bits = __builtin_bit_cast(uint16_t, (__bf16)v);
    return r;
}

__device__ __forceinline__ float fma_c(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
__device__ __forceinline__ double fma_c(double a, double b, double c) { return __builtin_fma(a, b, c); }

// VX consecutive storage elements, aligned so one vector load/store moves them.
template <typename S, int VX> struct alignas(sizeof(S) * VX) VecS {
    S v[VX];
};

// ---------------------------------------------------------------------------
// Whole-wavefront lane shifts (DPP wave_shr:1 / wave_shl:1).  Lane l receives
// the value of lane l-1 (shr) or l+1 (shl); with bound_ctrl set, the lane that
// has no source reads 0.
template <int CTRL> __device__ __forceinline__ float dpp32(float v) {
    return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), CTRL, 0xf, 0xf, true));
}
template <int CTRL> __device__ __forceinline__ double dpp32(double v) {
    const uint64_t u = (uint64_t)__double_as_longlong(v);
    const int lo = __builtin_amdgcn_mov_dpp((int)(uint32_t)u, CTRL, 0xf, 0xf, true);
    const int hi = __builtin_amdgcn_mov_dpp((int)(uint32_t)(u >> 32), CTRL, 0xf, 0xf, true);
    return __longlong_as_double((long long)(((uint64_t)(uint32_t)hi << 32) | (uint32_t)lo));
}
constexpr int kDppWaveShr1 = 0x138;  // from lane - 1
constexpr int kDppWaveShl1 = 0x130;  // from lane + 1

// value held by lane (l + S) of the wave (0 outside the wave)
template <int S, typename C> __device__ __forceinline__ C lane_shift(C v) {
    if constexpr (S == 0) {
        return v;
    } else if constexpr (S < 0) {
        return lane_shift<S + 1>(dpp32<kDppWaveShr1>(v));
    } else {
        return lane_shift<S - 1>(dpp32<kDppWaveShl1>(v));
    }
}

// ---------------------------------------------------------------------------
// Buffer (range-checked) loads and stores.  A resource covers one plane of a
// grid; offsets at or beyond its size read as 0 and drop stores, which is how
// the kernels handle points outside the grid without branches.
using rsrc_t = __amdgpu_buffer_rsrc_t;
constexpr int kBufferFlags = 0x00020000;  // raw 32-bit dword access (gfx9 family)
constexpr uint32_t kOutOfRange = 0x80000000u;  // byte offset beyond every resource

// The descriptor must live in scalar registers; its fields are uniform by
// construction, and readfirstlane says so to the compiler (a descriptor built
// from vector registers forces a loop over distinct values around every access).
__device__ __forceinline__ rsrc_t make_rsrc(const void *base, uint32_t bytes) {
    const uint64_t p = (uint64_t)base;
    const uint32_t lo = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)p);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)(p >> 32));
    const int n = __builtin_amdgcn_readfirstlane((int)bytes);
    void *q = (void *)(((uint64_t)hi << 32) | lo);
    return __builtin_amdgcn_make_buffer_rsrc(q, (short)0, n, kBufferFlags);
}

template <int BYTES> struct BufWord;
template <> struct BufWord<2> { using T = unsigned short; };
template <> struct BufWord<4> { using T = unsigned int; };
template <> struct BufWord<8> { using T = __attribute__((ext_vector_type(2))) unsigned int; };
template <> struct BufWord<16> { using T = __attribute__((ext_vector_type(4))) unsigned int; };

template <int BYTES> __device__ __forceinline__ typename BufWord<BYTES>::T buf_load(rsrc_t r, uint32_t off) {
    if constexpr (BYTES == 2) return __builtin_amdgcn_raw_buffer_load_b16(r, (int)off, 0, 0);
    if constexpr (BYTES == 4) return __builtin_amdgcn_raw_buffer_load_b32(r, (int)off, 0, 0);
    if constexpr (BYTES == 8) return __builtin_amdgcn_raw_buffer_load_b64(r, (int)off, 0, 0);
    if constexpr (BYTES == 16) return __builtin_amdgcn_raw_buffer_load_b128(r, (int)off, 0, 0);
}
template <int BYTES> __device__ __forceinline__ void buf_store(typename BufWord<BYTES>::T v, rsrc_t r, uint32_t off) {
    if constexpr (BYTES == 2) __builtin_amdgcn_raw_buffer_store_b16(v, r, (int)off, 0, 0);
    if constexpr (BYTES == 4) __builtin_amdgcn_raw_buffer_store_b32(v, r, (int)off, 0, 0);
    if constexpr (BYTES == 8) __builtin_amdgcn_raw_buffer_store_b64(v, r, (int)off, 0, 0);
    if constexpr (BYTES == 16) __builtin_amdgcn_raw_buffer_store_b128(v, r, (int)off, 0, 0);
}

// VX consecutive elements of type S through buffer instructions (<= 16 bytes per
// instruction; wider vectors are split)
template <typename S, int VX> __device__ __forceinline__ VecS<S, VX> vec_load(rsrc_t r, uint32_t off) {
    constexpr int B = (int)sizeof(S) * VX;
    if constexpr (B <= 16) {
        return __builtin_bit_cast(VecS<S, VX>, buf_load<B>(r, off));
    } else {
        VecS<S, VX> out;
        constexpr int H = VX / 2;
        const VecS<S, H> lo = vec_load<S, H>(r, off);
        const VecS<S, H> hi = vec_load<S, H>(r, off == kOutOfRange ? off : off + 16u);
#pragma unroll
        for (int v = 0; v < H; ++v) {
            out.v[v] = lo.v[v];
            out.v[H + v] = hi.v[v];
        }
        return out;
    }
}
template <typename S, int VX> __device__ __forceinline__ void vec_store(const VecS<S, VX> &t, rsrc_t r, uint32_t off) {
    constexpr int B = (int)sizeof(S) * VX;
    if constexpr (B <= 16) {
        buf_store<B>(__builtin_bit_cast(typename BufWord<B>::T, t), r, off);
    } else {
        constexpr int H = VX / 2;
        VecS<S, H> lo, hi;
#pragma unroll
        for (int v = 0; v < H; ++v) {
            lo.v[v] = t.v[v];
            hi.v[v] = t.v[H + v];
        }
        vec_store<S, H>(lo, r, off);
        vec_store<S, H>(hi, r, off == kOutOfRange ? off : off + 16u);
    }
}

// ---------------------------------------------------------------------------
// Compile-time loops: f(std::integral_constant<int, I>) for I in [B, E).
template <int B, int E, typename F> __device__ __forceinline__ void static_for(F &&f) {
    if constexpr (B < E) {
        f(std::integral_constant<int, B>{});
        static_for<B + 1, E>(f);
    }
}

// t[i] += c * (x[i] held by lane l + S) for N independent rows i, 0 outside
// the wave.  For FP32 the last one-lane step is a DPP operand of the FMA itself
// (v_fmac_f32 with a wave_shr:1 / wave_shl:1 source), so a neighbour in the
// adjacent lane costs one VALU instruction instead of a lane move plus an FMA;
// a source lane outside the wave reads 0 (bound_ctrl) and leaves t unchanged.
// The product is rounded once inside the fused multiply-add, exactly as in
// fma_c(c, x, t).  A DPP instruction must not read a register that a VALU
// instruction wrote in the two preceding wait states; the compiler's hazard
// pass does not look inside inline assembly, so each block of up to four
// instructions opens with its own s_nop (the instructions inside a block read
// no register another one of them writes: the outputs are early-clobber).
// FP64 uses lane moves (wave shifts are not available to 64-bit DPP operands).
#define STN_DPP_FMAC(D, X, C, CTL) "v_fmac_f32_dpp " D ", " X ", " C " " CTL " row_mask:0xf bank_mask:0xf bound_ctrl:1\n\t"
template <int S> __device__ __forceinline__ void dpp_fmac4(float c, const float *x, float *t) {
    static_assert(S == -1 || S == 1, "one-lane shift");
    if constexpr (S == -1) {
        asm("s_nop 1\n\t" STN_DPP_FMAC("%0", "%4", "%8", "wave_shr:1") STN_DPP_FMAC("%1", "%5", "%8", "wave_shr:1")
                STN_DPP_FMAC("%2", "%6", "%8", "wave_shr:1") STN_DPP_FMAC("%3", "%7", "%8", "wave_shr:1")
            : "+&v"(t[0]), "+&v"(t[1]), "+&v"(t[2]), "+&v"(t[3])
            : "v"(x[0]), "v"(x[1]), "v"(x[2]), "v"(x[3]), "v"(c));
    } else {
        asm("s_nop 1\n\t" STN_DPP_FMAC("%0", "%4", "%8", "wave_shl:1") STN_DPP_FMAC("%1", "%5", "%8", "wave_shl:1")
                STN_DPP_FMAC("%2", "%6", "%8", "wave_shl:1") STN_DPP_FMAC("%3", "%7", "%8", "wave_shl:1")
            : "+&v"(t[0]), "+&v"(t[1]), "+&v"(t[2]), "+&v"(t[3])
            : "v"(x[0]), "v"(x[1]), "v"(x[2]), "v"(x[3]), "v"(c));
    }
}
template <int S> __device__ __forceinline__ void dpp_fmac2(float c, const float *x, float *t) {
    static_assert(S == -1 || S == 1, "one-lane shift");
    if constexpr (S == -1) {
        asm("s_nop 1\n\t" STN_DPP_FMAC("%0", "%2", "%4", "wave_shr:1") STN_DPP_FMAC("%1", "%3", "%4", "wave_shr:1")
            : "+&v"(t[0]), "+&v"(t[1])
            : "v"(x[0]), "v"(x[1]), "v"(c));
    } else {
        asm("s_nop 1\n\t" STN_DPP_FMAC("%0", "%2", "%4", "wave_shl:1") STN_DPP_FMAC("%1", "%3", "%4", "wave_shl:1")
            : "+&v"(t[0]), "+&v"(t[1])
            : "v"(x[0]), "v"(x[1]), "v"(c));
    }
}
template <int S> __device__ __forceinline__ void dpp_fmac1(float c, const float *x, float *t) {
    static_assert(S == -1 || S == 1, "one-lane shift");
    if constexpr (S == -1) {
        asm("s_nop 1\n\t" STN_DPP_FMAC("%0", "%1", "%2", "wave_shr:1")
            : "+&v"(t[0])
            : "v"(x[0]), "v"(c));
    } else {
        asm("s_nop 1\n\t" STN_DPP_FMAC("%0", "%1", "%2", "wave_shl:1")
            : "+&v"(t[0])
            : "v"(x[0]), "v"(c));
    }
}

// acc += (x[i] held by lane l + S) * u[i] for i = 0 .. N-1 in that order: one
// accumulator, the lane-shifted operand a DPP source as in fma_shift_rows (a
// source lane outside the wave reads 0).  The instructions of a block write
// only acc, which no DPP operand reads, so one s_nop per block covers the
// hazard on the x registers.
template <int S, int N> __device__ __forceinline__ void dpp_fmac_chain(const float (&u)[N], const float (&x)[N], float &acc) {
    static_assert(S == -1 || S == 1, "one-lane shift");
    constexpr int N4 = N / 4 * 4;
#pragma unroll
    for (int b = 0; b < N4; b += 4) {
        if constexpr (S == -1)
            asm("s_nop 1\n\t" STN_DPP_FMAC("%0", "%1", "%5", "wave_shr:1") STN_DPP_FMAC("%0", "%2", "%6", "wave_shr:1")
                    STN_DPP_FMAC("%0", "%3", "%7", "wave_shr:1") STN_DPP_FMAC("%0", "%4", "%8", "wave_shr:1")
                : "+v"(acc)
                : "v"(x[b]), "v"(x[b + 1]), "v"(x[b + 2]), "v"(x[b + 3]), "v"(u[b]), "v"(u[b + 1]), "v"(u[b + 2]),
                  "v"(u[b + 3]));
        else
            asm("s_nop 1\n\t" STN_DPP_FMAC("%0", "%1", "%5", "wave_shl:1") STN_DPP_FMAC("%0", "%2", "%6", "wave_shl:1")
                    STN_DPP_FMAC("%0", "%3", "%7", "wave_shl:1") STN_DPP_FMAC("%0", "%4", "%8", "wave_shl:1")
                : "+v"(acc)
                : "v"(x[b]), "v"(x[b + 1]), "v"(x[b + 2]), "v"(x[b + 3]), "v"(u[b]), "v"(u[b + 1]), "v"(u[b + 2]),
                  "v"(u[b + 3]));
    }
#pragma unroll
    for (int i = N4; i < N; ++i) {
        if constexpr (S == -1)
            asm("s_nop 1\n\t" STN_DPP_FMAC("%0", "%1", "%2", "wave_shr:1") : "+v"(acc) : "v"(x[i]), "v"(u[i]));
        else
            asm("s_nop 1\n\t" STN_DPP_FMAC("%0", "%1", "%2", "wave_shl:1") : "+v"(acc) : "v"(x[i]), "v"(u[i]));
    }
}
#undef STN_DPP_FMAC

template <int S, int N> __device__ __forceinline__ void fma_shift_rows(float c, const float (&x)[N], float (&t)[N]) {
    static_assert(S != 0, "no shift");
    if constexpr (S < -1 || S > 1) {
        float y[N];
#pragma unroll
        for (int i = 0; i < N; ++i) y[i] = dpp32<(S < 0) ? kDppWaveShr1 : kDppWaveShl1>(x[i]);
        fma_shift_rows<(S < 0) ? S + 1 : S - 1, N>(c, y, t);
    } else {
        constexpr int S1 = S;
        static_for<0, N / 4>([&](auto B_) { dpp_fmac4<S1>(c, x + 4 * decltype(B_)::value, t + 4 * decltype(B_)::value); });
        constexpr int done = N / 4 * 4;
        if constexpr (N - done >= 2) dpp_fmac2<S1>(c, x + done, t + done);
        if constexpr ((N - done) % 2 == 1) dpp_fmac1<S1>(c, x + N - 1, t + N - 1);
    }
}
template <int S, int N> __device__ __forceinline__ void fma_shift_rows(double c, const double (&x)[N], double (&t)[N]) {
#pragma unroll
    for (int i = 0; i < N; ++i) t[i] = fma_c(c, lane_shift<S>(x[i]), t[i]);
}


// Masks built with integer arithmetic (-1 = true, 0 = false), so wave-uniform
// tests stay in scalar registers: a comparison turned into a bool becomes a
// lane mask, and selecting with it costs a vector instruction per use.
__device__ __forceinline__ int mask_lt(int a, int b) { return (a - b) >> 31; }  // a < b (no overflow)
__device__ __forceinline__ int mask_in(int v, int n) { return ~((v | (n - 1 - v)) >> 31); }  // 0 <= v < n
// bitwise OR of two values (one of them +0.0): the other value, exactly
__device__ __forceinline__ float bits_or(float a, float b) { return __int_as_float(__float_as_int(a) | __float_as_int(b)); }
__device__ __forceinline__ double bits_or(double a, double b) {
    return __longlong_as_double(__double_as_longlong(a) | __double_as_longlong(b));
}
__device__ __forceinline__ float weight_if(float c, int mask) { return __int_as_float(__float_as_int(c) & mask); }
__device__ __forceinline__ double weight_if(double c, int mask) {
    return __longlong_as_double(__double_as_longlong(c) & (long long)mask);  // mask sign-extends
}

constexpr int floordiv(int a, int b) { return (a >= 0) ? a / b : -((-a + b - 1) / b); }
constexpr int posmod(int a, int b) { return ((a % b) + b) % b; }

// ---------------------------------------------------------------------------
// Workgroups are dispatched round-robin over the 8 XCDs (each with its own L2).
// Remap the hardware block id so every XCD gets a contiguous range of
// logical tiles; neighbouring tiles then share halo reads through one L2.
constexpr int kNumXcd = 8;
__device__ __forceinline__ int xcd_remap(int b, int n) {
    const int q = n / kNumXcd, rem = n % kNumXcd;
    const int xcd = b % kNumXcd, idx = b / kNumXcd;
    return xcd < rem ? xcd * (q + 1) + idx : rem * (q + 1) + (xcd - rem) * q + idx;
}

__device__ __forceinline__ int64_t wrap_index(int64_t i, int64_t n) {
    int64_t m = i % n;
    return m < 0 ? m + n : m;
}

}  // namespace stn
