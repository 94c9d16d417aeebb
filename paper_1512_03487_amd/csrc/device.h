// Device building blocks for the hopping-term kernels (gfx950, wave64).
//
// * Cx<C>: a complex number in the compute precision C (double or float).
// * Spinor storage policies SpF64 / SpF32 / SpF16S: load a site's 4x3 complex spinor (or one
//   chiral half of it) into registers in precision C and store it back, with the per-site scale
//   of the FP16 format applied on load and computed on store. Stores are plain: the L2 merges
//   a wave's partial-line writes, whereas streaming stores of 16-byte pieces at the 96/192-byte
//   site pitch were measured to double the HBM write traffic.
// * Link storage policies: 18-real or 12-real (row 2 rebuilt as conj(row0 x row1)) in double,
//   float or half.
// * Spin projection to a two-spin half-spinor and its reconstruction, specialised per direction
//   (the Compressor's spin projection of Section 2.4 done on load).
// * Geometry: coordinates of a linear site and its periodic neighbours (Cshift semantics of
//   Section 2.3), plus the XCD-aware block order.
#pragma once

#include <hip/hip_runtime.h>
#include <hip/hip_fp16.h>
#include <stdint.h>

#include <type_traits>

namespace gridmi {

template <typename C>
struct Cx {
    C r, i;
};

template <typename C>
__device__ __forceinline__ Cx<C> cadd(Cx<C> a, Cx<C> b) { return {a.r + b.r, a.i + b.i}; }
template <typename C>
__device__ __forceinline__ Cx<C> csub(Cx<C> a, Cx<C> b) { return {a.r - b.r, a.i - b.i}; }
// a * b
template <typename C>
__device__ __forceinline__ Cx<C> cmul(Cx<C> a, Cx<C> b) { return {a.r * b.r - a.i * b.i, a.r * b.i + a.i * b.r}; }
// conj(a) * b
template <typename C>
__device__ __forceinline__ Cx<C> cmulc(Cx<C> a, Cx<C> b) { return {a.r * b.r + a.i * b.i, a.r * b.i - a.i * b.r}; }
// acc + a * b
template <typename C>
__device__ __forceinline__ Cx<C> cmac(Cx<C> acc, Cx<C> a, Cx<C> b) {
    return {acc.r + a.r * b.r - a.i * b.i, acc.i + a.r * b.i + a.i * b.r};
}
// acc + conj(a) * b
template <typename C>
__device__ __forceinline__ Cx<C> cmacc(Cx<C> acc, Cx<C> a, Cx<C> b) {
    return {acc.r + a.r * b.r + a.i * b.i, acc.i + a.r * b.i - a.i * b.r};
}
// i * a
template <typename C>
__device__ __forceinline__ Cx<C> ctimesi(Cx<C> a) { return {-a.i, a.r}; }
template <typename C>
__device__ __forceinline__ Cx<C> cscale(C s, Cx<C> a) { return {s * a.r, s * a.i}; }
template <typename C>
__device__ __forceinline__ Cx<C> cconj(Cx<C> a) { return {a.r, -a.i}; }

// ------------------------------------------------------------------------------------------
// Spinor storage. A site is 12 complex numbers [spin][colour]; `site` counts sites (4D or 5D).
// ------------------------------------------------------------------------------------------

struct SpF64 {
    using C = double;
    static constexpr int kBytes = 192;
    static constexpr int kChunks = 12;          // 16-byte chunks per site
    static constexpr bool kScaled = false;
    __device__ __forceinline__ static void unpack(const uint4 *w, float, Cx<C> p[4][3]) {
#pragma unroll
        for (int k = 0; k < 12; ++k) {
            double2 v;
            __builtin_memcpy(&v, &w[k], 16);
            p[k / 3][k % 3] = {v.x, v.y};
        }
    }
    __device__ __forceinline__ static void load(const void *base, const float *, size_t site, Cx<C> p[4][3]) {
        const double2 *q = reinterpret_cast<const double2 *>(base) + site * 12;
#pragma unroll
        for (int k = 0; k < 12; ++k) {
            double2 v = q[k];
            p[k / 3][k % 3] = {v.x, v.y};
        }
    }
    // spins (2h, 2h+1): h = 0 upper (P_+), h = 1 lower (P_-)
    __device__ __forceinline__ static void load_half(const void *base, const float *, size_t site, int h,
                                                     Cx<C> p[2][3]) {
        const double2 *q = reinterpret_cast<const double2 *>(base) + site * 12 + h * 6;
#pragma unroll
        for (int k = 0; k < 6; ++k) {
            double2 v = q[k];
            p[k / 3][k % 3] = {v.x, v.y};
        }
    }
    __device__ __forceinline__ static void store(void *base, float *, size_t site, const Cx<C> p[4][3]) {
        double2 *q = reinterpret_cast<double2 *>(base) + site * 12;
#pragma unroll
        for (int k = 0; k < 12; ++k) q[k] = make_double2(p[k / 3][k % 3].r, p[k / 3][k % 3].i);
    }
    // store, returning the squared norm of the stored site
    __device__ __forceinline__ static double store_n2(void *base, float *scale, size_t site, const Cx<C> p[4][3]) {
        store(base, scale, site, p);
        double n = 0.0;
#pragma unroll
        for (int k = 0; k < 12; ++k) n += p[k / 3][k % 3].r * p[k / 3][k % 3].r + p[k / 3][k % 3].i * p[k / 3][k % 3].i;
        return n;
    }
};

struct SpF32 {
    using C = float;
    static constexpr int kBytes = 96;
    static constexpr int kChunks = 6;
    static constexpr bool kScaled = false;
    __device__ __forceinline__ static void unpack(const uint4 *w, float, Cx<C> p[4][3]) {
#pragma unroll
        for (int k = 0; k < 6; ++k) {
            float4 v;
            __builtin_memcpy(&v, &w[k], 16);
            p[(2 * k) / 3][(2 * k) % 3] = {v.x, v.y};
            p[(2 * k + 1) / 3][(2 * k + 1) % 3] = {v.z, v.w};
        }
    }
    __device__ __forceinline__ static void load(const void *base, const float *, size_t site, Cx<C> p[4][3]) {
        const float4 *q = reinterpret_cast<const float4 *>(base) + site * 6;
#pragma unroll
        for (int k = 0; k < 6; ++k) {
            float4 v = q[k];
            p[(2 * k) / 3][(2 * k) % 3] = {v.x, v.y};
            p[(2 * k + 1) / 3][(2 * k + 1) % 3] = {v.z, v.w};
        }
    }
    __device__ __forceinline__ static void load_half(const void *base, const float *, size_t site, int h,
                                                     Cx<C> p[2][3]) {
        const float4 *q = reinterpret_cast<const float4 *>(base) + site * 6 + h * 3;
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            float4 v = q[k];
            p[(2 * k) / 3][(2 * k) % 3] = {v.x, v.y};
            p[(2 * k + 1) / 3][(2 * k + 1) % 3] = {v.z, v.w};
        }
    }
    __device__ __forceinline__ static void store(void *base, float *, size_t site, const Cx<C> p[4][3]) {
        float4 *q = reinterpret_cast<float4 *>(base) + site * 6;
#pragma unroll
        for (int k = 0; k < 6; ++k) {
            const Cx<C> a = p[(2 * k) / 3][(2 * k) % 3], b = p[(2 * k + 1) / 3][(2 * k + 1) % 3];
            q[k] = make_float4(a.r, a.i, b.r, b.i);
        }
    }
    __device__ __forceinline__ static double store_n2(void *base, float *scale, size_t site, const Cx<C> p[4][3]) {
        store(base, scale, site, p);
        double n = 0.0;
#pragma unroll
        for (int k = 0; k < 12; ++k) {
            const double r = p[k / 3][k % 3].r, i = p[k / 3][k % 3].i;
            n += r * r + i * i;
        }
        return n;
    }
};

__device__ __forceinline__ float half_bits_to_float(uint32_t bits16) {
    return __half2float(__ushort_as_half(static_cast<unsigned short>(bits16)));
}
__device__ __forceinline__ uint32_t float_to_half_bits(float v) {
    return static_cast<uint32_t>(__half_as_ushort(__float2half_rn(v)));
}
// half(v * r) with the product first rounded to float: the FP16 code is defined by two roundings,
// so the multiply must not be fused into a mixed-precision FMA that rounds once.
// The empty asm only pins the float product in a register (an optimisation barrier; no memory
// access), which stops instruction selection from fusing the multiply into the conversion.
__device__ __forceinline__ uint32_t scaled_half_bits(float v, float r) {
    float p = v * r;
    __asm__ volatile("" : "+v"(p));
    return float_to_half_bits(p);
}

// FP16 storage: 24 halves (48 bytes) per site and one float scale per site.
struct SpF16S {
    using C = float;
    static constexpr int kBytes = 52;
    static constexpr int kChunks = 3;
    static constexpr bool kScaled = true;
    __device__ __forceinline__ static void unpack(const uint4 *w, float s, Cx<C> p[4][3]) {
        unpack6(w[0], w[1], w[2], s, p);
    }
    __device__ __forceinline__ static void unpack6(uint4 w0, uint4 w1, uint4 w2, float s, Cx<C> p[4][3]) {
        const uint32_t w[12] = {w0.x, w0.y, w0.z, w0.w, w1.x, w1.y, w1.z, w1.w, w2.x, w2.y, w2.z, w2.w};
#pragma unroll
        for (int k = 0; k < 12; ++k)
            p[k / 3][k % 3] = {half_bits_to_float(w[k] & 0xffffu) * s, half_bits_to_float(w[k] >> 16) * s};
    }
    __device__ __forceinline__ static void load(const void *base, const float *scale, size_t site, Cx<C> p[4][3]) {
        const uint4 *q = reinterpret_cast<const uint4 *>(base) + site * 3;
        const float s = scale[site];
        unpack6(q[0], q[1], q[2], s, p);
    }
    __device__ __forceinline__ static void load_half(const void *base, const float *scale, size_t site, int h,
                                                     Cx<C> p[2][3]) {
        // a half site is 6 complex = 24 bytes: 3 x 8-byte words
        const uint2 *q = reinterpret_cast<const uint2 *>(base) + site * 6 + h * 3;
        const float s = scale[site];
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            uint2 v = q[k];
            p[(2 * k) / 3][(2 * k) % 3] = {half_bits_to_float(v.x & 0xffffu) * s, half_bits_to_float(v.x >> 16) * s};
            p[(2 * k + 1) / 3][(2 * k + 1) % 3] = {half_bits_to_float(v.y & 0xffffu) * s,
                                                  half_bits_to_float(v.y >> 16) * s};
        }
    }
    __device__ __forceinline__ static float encode(const Cx<C> p[4][3], uint32_t w[12]) {
        float m = 0.f;
#pragma unroll
        for (int k = 0; k < 12; ++k) m = fmaxf(m, fmaxf(fabsf(p[k / 3][k % 3].r), fabsf(p[k / 3][k % 3].i)));
        const float inv = m > 0.f ? 1.0f / m : 0.f;
#pragma unroll
        for (int k = 0; k < 12; ++k) {
            w[k] = scaled_half_bits(p[k / 3][k % 3].r, inv) | (scaled_half_bits(p[k / 3][k % 3].i, inv) << 16);
        }
        return m;
    }
    __device__ __forceinline__ static void put(void *base, float *scale, size_t site, const uint32_t w[12], float m) {
        uint4 *q = reinterpret_cast<uint4 *>(base) + site * 3;
        q[0] = make_uint4(w[0], w[1], w[2], w[3]);
        q[1] = make_uint4(w[4], w[5], w[6], w[7]);
        q[2] = make_uint4(w[8], w[9], w[10], w[11]);
        scale[site] = m;
    }
    __device__ __forceinline__ static void store(void *base, float *scale, size_t site, const Cx<C> p[4][3]) {
        uint32_t w[12];
        const float m = encode(p, w);
        put(base, scale, site, w, m);
    }
    // store, returning the squared norm of the stored (coded) site
    __device__ __forceinline__ static double store_n2(void *base, float *scale, size_t site, const Cx<C> p[4][3]) {
        uint32_t w[12];
        const float m = encode(p, w);
        put(base, scale, site, w, m);
        double n = 0.0;
#pragma unroll
        for (int k = 0; k < 12; ++k) {
            const double r = half_bits_to_float(w[k] & 0xffffu) * m, i = half_bits_to_float(w[k] >> 16) * m;
            n += r * r + i * i;
        }
        return n;
    }
};

// ------------------------------------------------------------------------------------------
// Reductions inside one 16-lane DPP row / one wavefront with DPP moves (VALU) instead of the
// LDS-path lane permutes. Each step pairs a lane with one of the other group: xor 1 and xor 2
// (quad_perm [1,0,3,2] and [2,3,0,1]), then the mirror inside each half-row and inside the row,
// after which every lane of the row holds the row's result. All lanes must be active.
// ------------------------------------------------------------------------------------------

template <int CTRL>
__device__ __forceinline__ float dpp_f32(float v) {
    return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), CTRL, 0xf, 0xf, false));
}
template <int CTRL>
__device__ __forceinline__ double dpp_f64(double v) {
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_mov_dpp(static_cast<int>(b), CTRL, 0xf, 0xf, false);
    const int hi = __builtin_amdgcn_mov_dpp(static_cast<int>(b >> 32), CTRL, 0xf, 0xf, false);
    return __longlong_as_double((static_cast<long long>(hi) << 32) | static_cast<unsigned int>(lo));
}
constexpr int kDppXor1 = 0xB1, kDppXor2 = 0x4E, kDppHalfMirror = 0x141, kDppMirror = 0x140;

// max over the 16 lanes of each row (exact: any pairing order gives the same maximum)
__device__ __forceinline__ float row_max16(float m) {
    m = fmaxf(m, dpp_f32<kDppXor1>(m));
    m = fmaxf(m, dpp_f32<kDppXor2>(m));
    m = fmaxf(m, dpp_f32<kDppHalfMirror>(m));
    return fmaxf(m, dpp_f32<kDppMirror>(m));
}

// sum over the wavefront, in a fixed order (the same in every lane and every run)
__device__ __forceinline__ double wave_sum64(double v) {
    v += dpp_f64<kDppXor1>(v);
    v += dpp_f64<kDppXor2>(v);
    v += dpp_f64<kDppHalfMirror>(v);
    v += dpp_f64<kDppMirror>(v);
    auto lane_val = [&](int l) {
        const long long b = __double_as_longlong(v);
        const int lo = __builtin_amdgcn_readlane(static_cast<int>(b), l);
        const int hi = __builtin_amdgcn_readlane(static_cast<int>(b >> 32), l);
        return __longlong_as_double((static_cast<long long>(hi) << 32) | static_cast<unsigned int>(lo));
    };
    return (lane_val(0) + lane_val(16)) + (lane_val(32) + lane_val(48));
}

// ------------------------------------------------------------------------------------------
// Per-component access to a spinor record (used where lanes own components, not sites).
// ------------------------------------------------------------------------------------------

// Complex number k (spin k / 3, colour k % 3) of a record: staged in LDS or in global memory.
template <class SP>
struct Elem;

template <>
struct Elem<SpF64> {
    __device__ __forceinline__ static Cx<double> get(const void *rec, int k, float) {
        const double2 v = reinterpret_cast<const double2 *>(rec)[k];
        return {v.x, v.y};
    }
};
template <>
struct Elem<SpF32> {
    __device__ __forceinline__ static Cx<float> get(const void *rec, int k, float) {
        const float2 v = reinterpret_cast<const float2 *>(rec)[k];
        return {v.x, v.y};
    }
};
template <>
struct Elem<SpF16S> {
    __device__ __forceinline__ static Cx<float> get(const void *rec, int k, float s) {
        const uint32_t w = reinterpret_cast<const uint32_t *>(rec)[k];
        return {half_bits_to_float(w & 0xffffu) * s, half_bits_to_float(w >> 16) * s};
    }
};

template <class SP>
__device__ __forceinline__ Cx<typename SP::C> global_elem(const void *base, const float *scale, size_t rec, int k) {
    const char *p = reinterpret_cast<const char *>(base) + rec * (SP::kChunks * 16);
    return Elem<SP>::get(p, k, SP::kScaled ? scale[rec] : 1.0f);
}

// Store complex k of record rec, non-temporal (the output is not re-read by the kernel; keeping
// it out of L2 leaves room for the inputs' reuse, measured 3-10 % faster). FP16 storage: the 16
// lanes of a site (12 active) agree on the site scale max |re|, |im| before encoding.
typedef double ntd2 __attribute__((ext_vector_type(2)));
typedef float ntf2 __attribute__((ext_vector_type(2)));
template <class SP>
__device__ __forceinline__ void store_elem(void *base, float *scale, size_t rec, int k, Cx<typename SP::C> v, bool live);

template <>
__device__ __forceinline__ void store_elem<SpF64>(void *base, float *, size_t rec, int k, Cx<double> v, bool live) {
    if (live) {
        const ntd2 w = {v.r, v.i};
        __builtin_nontemporal_store(w, reinterpret_cast<ntd2 *>(base) + rec * 12 + k);
    }
}
template <>
__device__ __forceinline__ void store_elem<SpF32>(void *base, float *, size_t rec, int k, Cx<float> v, bool live) {
    if (live) {
        const ntf2 w = {v.r, v.i};
        __builtin_nontemporal_store(w, reinterpret_cast<ntf2 *>(base) + rec * 12 + k);
    }
}
template <>
__device__ __forceinline__ void store_elem<SpF16S>(void *base, float *scale, size_t rec, int k, Cx<float> v, bool live) {
    const float m = row_max16(live ? fmaxf(fabsf(v.r), fabsf(v.i)) : 0.f);
    const float inv = m > 0.f ? 1.0f / m : 0.f;
    const uint32_t w = scaled_half_bits(v.r, inv) | (scaled_half_bits(v.i, inv) << 16);
    if (live) {
        reinterpret_cast<uint32_t *>(base)[rec * 12 + k] = w;
        if (k == 0) scale[rec] = m;
    }
}

// |v|^2 of complex k as store_elem will store it (0 for idle lanes; FP16 storage: of the coded
// value, with the same site scale), without storing: a block can reduce it before its stores.
template <class SP>
__device__ __forceinline__ double stored_n2(Cx<typename SP::C> v, bool live) {
    return live ? double(v.r) * double(v.r) + double(v.i) * double(v.i) : 0.0;
}
template <>
__device__ __forceinline__ double stored_n2<SpF16S>(Cx<float> v, bool live) {
    const float m = row_max16(live ? fmaxf(fabsf(v.r), fabsf(v.i)) : 0.f);
    const float inv = m > 0.f ? 1.0f / m : 0.f;
    const uint32_t w = scaled_half_bits(v.r, inv) | (scaled_half_bits(v.i, inv) << 16);
    const double r = half_bits_to_float(w & 0xffffu) * m, i = half_bits_to_float(w >> 16) * m;
    return live ? r * r + i * i : 0.0;
}

// ------------------------------------------------------------------------------------------
// Link storage. `link` = site * 4 + mu. Loads fill u[3][3] (row 2 rebuilt for 12-real links).
// ------------------------------------------------------------------------------------------

template <typename C>
__device__ __forceinline__ void rebuild_row2(Cx<C> u[3][3]) {
    // row2 = conj(row0 x row1)
    u[2][0] = cconj(csub(cmul(u[0][1], u[1][2]), cmul(u[0][2], u[1][1])));
    u[2][1] = cconj(csub(cmul(u[0][2], u[1][0]), cmul(u[0][0], u[1][2])));
    u[2][2] = cconj(csub(cmul(u[0][0], u[1][1]), cmul(u[0][1], u[1][0])));
}

// Split link load for kernels in which lanes l and l + 32 of a wavefront need the same link: the
// two half-wavefronts load alternate elements, so one load instruction reads each link's bytes
// once instead of twice, and v_permlane32_swap (gfx950) exchanges them: with both operands equal
// to x it returns [x(lanes 0-31) | x(lanes 0-31)] and [x(lanes 32-63) | x(lanes 32-63)].
// issue() only loads; finish() exchanges, so the loads can be in flight across other work.
template <class E, int N>
struct SplitLoad {
    static_assert(sizeof(E) % 4 == 0, "element of whole dwords");
    static constexpr int NP = N / 2, W = sizeof(E) / 4;
    E v[NP + (N & 1)];
    __device__ __forceinline__ void issue(const E *__restrict__ q, int half) {
#pragma unroll
        for (int m = 0; m < NP; ++m) v[m] = q[2 * m + half];
        if (N & 1) v[NP] = q[N - 1];
    }
    __device__ __forceinline__ void finish(E out[N]) const {
#pragma unroll
        for (int m = 0; m < NP; ++m) {
            uint32_t d[W], lo[W], hi[W];
            __builtin_memcpy(d, &v[m], sizeof(E));
#pragma unroll
            for (int w = 0; w < W; ++w) {
                const auto r = __builtin_amdgcn_permlane32_swap(d[w], d[w], false, false);
                lo[w] = r[0];
                hi[w] = r[1];
            }
            __builtin_memcpy(&out[2 * m], lo, sizeof(E));
            __builtin_memcpy(&out[2 * m + 1], hi, sizeof(E));
        }
        if (N & 1) out[N - 1] = v[NP];
    }
};

template <int ROWS>
struct LkF64 {
    using C = double;
    static constexpr int kRows = ROWS;
    static constexpr int kBytes = ROWS * 3 * 16;
    __device__ __forceinline__ static void load(const void *base, size_t link, Cx<C> u[3][3]) {
        const double2 *q = reinterpret_cast<const double2 *>(base) + link * (ROWS * 3);
#pragma unroll
        for (int k = 0; k < ROWS * 3; ++k) {
            double2 v = q[k];
            u[k / 3][k % 3] = {v.x, v.y};
        }
        if (ROWS == 2) rebuild_row2(u);
    }
    // raw elements of a link and their decoding (for SplitLoad)
    using E = double2;
    static constexpr int kN = ROWS * 3;
    __device__ __forceinline__ static const E *elems(const void *base, size_t link) {
        return reinterpret_cast<const E *>(base) + link * kN;
    }
    __device__ __forceinline__ static void decode(const E e[kN], Cx<C> u[3][3]) {
#pragma unroll
        for (int k = 0; k < kN; ++k) u[k / 3][k % 3] = {e[k].x, e[k].y};
        if (ROWS == 2) rebuild_row2(u);
    }
};

template <int ROWS>
struct LkF32 {
    using C = float;
    static constexpr int kRows = ROWS;
    static constexpr int kBytes = ROWS * 3 * 8;
    __device__ __forceinline__ static void load(const void *base, size_t link, Cx<C> u[3][3]) {
        if (ROWS == 2) {
            const float4 *q = reinterpret_cast<const float4 *>(base) + link * 3;
#pragma unroll
            for (int k = 0; k < 3; ++k) {
                float4 v = q[k];
                u[(2 * k) / 3][(2 * k) % 3] = {v.x, v.y};
                u[(2 * k + 1) / 3][(2 * k + 1) % 3] = {v.z, v.w};
            }
            rebuild_row2(u);
        } else {
            const float2 *q = reinterpret_cast<const float2 *>(base) + link * 9;
#pragma unroll
            for (int k = 0; k < 9; ++k) {
                float2 v = q[k];
                u[k / 3][k % 3] = {v.x, v.y};
            }
        }
    }
};

template <int ROWS>
struct LkF16 {
    using C = float;
    static constexpr int kRows = ROWS;
    static constexpr int kBytes = ROWS * 3 * 4;
    __device__ __forceinline__ static void load(const void *base, size_t link, Cx<C> u[3][3]) {
        if (ROWS == 2) {
            const uint2 *q = reinterpret_cast<const uint2 *>(base) + link * 3;
#pragma unroll
            for (int k = 0; k < 3; ++k) {
                uint2 v = q[k];
                u[(2 * k) / 3][(2 * k) % 3] = {half_bits_to_float(v.x & 0xffffu), half_bits_to_float(v.x >> 16)};
                u[(2 * k + 1) / 3][(2 * k + 1) % 3] = {half_bits_to_float(v.y & 0xffffu),
                                                      half_bits_to_float(v.y >> 16)};
            }
            rebuild_row2(u);
        } else {
            const uint32_t *q = reinterpret_cast<const uint32_t *>(base) + link * 9;
#pragma unroll
            for (int k = 0; k < 9; ++k) {
                uint32_t v = q[k];
                u[k / 3][k % 3] = {half_bits_to_float(v & 0xffffu), half_bits_to_float(v >> 16)};
            }
        }
    }
};

// ------------------------------------------------------------------------------------------
// Spin projection (1 + EPS gamma_MU) psi = [h; EPS A_MU^dagger h], h = psi_up + EPS A_MU psi_dn,
// with gamma_MU = [[0, A], [A^dagger, 0]], A = -i sigma_1, -i sigma_2, -i sigma_3, 1.
// ------------------------------------------------------------------------------------------

template <int MU, int EPS, typename C>
__device__ __forceinline__ void project(const Cx<C> p[4][3], Cx<C> h[2][3]) {
    const C e = static_cast<C>(EPS);
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        if (MU == 0) {          // h0 = p0 - i e p3, h1 = p1 - i e p2
            h[0][a] = {p[0][a].r + e * p[3][a].i, p[0][a].i - e * p[3][a].r};
            h[1][a] = {p[1][a].r + e * p[2][a].i, p[1][a].i - e * p[2][a].r};
        } else if (MU == 1) {   // h0 = p0 - e p3, h1 = p1 + e p2
            h[0][a] = {p[0][a].r - e * p[3][a].r, p[0][a].i - e * p[3][a].i};
            h[1][a] = {p[1][a].r + e * p[2][a].r, p[1][a].i + e * p[2][a].i};
        } else if (MU == 2) {   // h0 = p0 - i e p2, h1 = p1 + i e p3
            h[0][a] = {p[0][a].r + e * p[2][a].i, p[0][a].i - e * p[2][a].r};
            h[1][a] = {p[1][a].r - e * p[3][a].i, p[1][a].i + e * p[3][a].r};
        } else {                // h0 = p0 + e p2, h1 = p1 + e p3
            h[0][a] = {p[0][a].r + e * p[2][a].r, p[0][a].i + e * p[2][a].i};
            h[1][a] = {p[1][a].r + e * p[3][a].r, p[1][a].i + e * p[3][a].i};
        }
    }
}

// acc += [chi; EPS A_MU^dagger chi]
template <int MU, int EPS, typename C>
__device__ __forceinline__ void reconstruct_add(Cx<C> acc[4][3], const Cx<C> chi[2][3]) {
    const C e = static_cast<C>(EPS);
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        acc[0][a] = cadd(acc[0][a], chi[0][a]);
        acc[1][a] = cadd(acc[1][a], chi[1][a]);
        if (MU == 0) {          // lower = (i e chi1, i e chi0)
            acc[2][a] = {acc[2][a].r - e * chi[1][a].i, acc[2][a].i + e * chi[1][a].r};
            acc[3][a] = {acc[3][a].r - e * chi[0][a].i, acc[3][a].i + e * chi[0][a].r};
        } else if (MU == 1) {   // lower = (e chi1, -e chi0)
            acc[2][a] = {acc[2][a].r + e * chi[1][a].r, acc[2][a].i + e * chi[1][a].i};
            acc[3][a] = {acc[3][a].r - e * chi[0][a].r, acc[3][a].i - e * chi[0][a].i};
        } else if (MU == 2) {   // lower = (i e chi0, -i e chi1)
            acc[2][a] = {acc[2][a].r - e * chi[0][a].i, acc[2][a].i + e * chi[0][a].r};
            acc[3][a] = {acc[3][a].r + e * chi[1][a].i, acc[3][a].i - e * chi[1][a].r};
        } else {                // lower = (e chi0, e chi1)
            acc[2][a] = {acc[2][a].r + e * chi[0][a].r, acc[2][a].i + e * chi[0][a].i};
            acc[3][a] = {acc[3][a].r + e * chi[1][a].r, acc[3][a].i + e * chi[1][a].i};
        }
    }
}

// chi_k = U h_k
template <typename C>
__device__ __forceinline__ void su3_mul(const Cx<C> u[3][3], const Cx<C> h[2][3], Cx<C> chi[2][3]) {
#pragma unroll
    for (int k = 0; k < 2; ++k)
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            Cx<C> s = cmul(u[a][0], h[k][0]);
            s = cmac(s, u[a][1], h[k][1]);
            s = cmac(s, u[a][2], h[k][2]);
            chi[k][a] = s;
        }
}

// chi_k = U^dagger h_k
template <typename C>
__device__ __forceinline__ void su3_adj_mul(const Cx<C> u[3][3], const Cx<C> h[2][3], Cx<C> chi[2][3]) {
#pragma unroll
    for (int k = 0; k < 2; ++k)
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            Cx<C> s = cmulc(u[0][a], h[k][0]);
            s = cmacc(s, u[1][a], h[k][1]);
            s = cmacc(s, u[2][a], h[k][2]);
            chi[k][a] = s;
        }
}

// Pin the accumulator in registers at this point of the program. The only use of the result is
// the store of live lanes, so without this the compiler sinks all arithmetic below the last
// gather (which every lane must execute) and keeps every gathered record live at once.
template <typename C>
__device__ __forceinline__ void pin(Cx<C> a[4][3]) {
#pragma unroll
    for (int j = 0; j < 12; ++j) __asm__ volatile("" : "+v"(a[j / 3][j % 3].r), "+v"(a[j / 3][j % 3].i));
}

// acc += (1 + E gamma_MU) V psi with V = U (ADJ false) or U^dagger (ADJ true)
template <int MU, int E, bool ADJ, typename C>
__device__ __forceinline__ void hop_term(Cx<C> acc[4][3], const Cx<C> p[4][3], const Cx<C> u[3][3]) {
    Cx<C> h[2][3], chi[2][3];
    project<MU, E>(p, h);
    if (ADJ)
        su3_adj_mul(u, h, chi);
    else
        su3_mul(u, h, chi);
    reconstruct_add<MU, E>(acc, chi);
    pin(acc);
    // One direction at a time: hoisting later directions' loads above this point would raise
    // per-wave parallelism at a larger cost in occupancy.
    __builtin_amdgcn_sched_barrier(0);
}

// ------------------------------------------------------------------------------------------
// Geometry
// ------------------------------------------------------------------------------------------

struct GeomDev {
    int L[4];        // Lx, Ly, Lz, Lt
    int Ls;          // fifth extent (1 for 4D)
    int vol;         // 4D volume
    int n5;          // vol * Ls
};

// Coordinates of 4D site x4 and the linear indices of its 8 periodic neighbours:
// nb[2 mu] = x + mu-hat, nb[2 mu + 1] = x - mu-hat.
__device__ __forceinline__ void neighbours(const GeomDev &g, int x4, int nb[8]) {
    int r = x4;
    int stride = 1;
#pragma unroll
    for (int mu = 0; mu < 4; ++mu) {
        const int L = g.L[mu];
        const int c = (mu < 3) ? r % L : r;
        r = (mu < 3) ? r / L : 0;
        nb[2 * mu] = x4 + ((c == L - 1) ? (1 - L) * stride : stride);
        nb[2 * mu + 1] = x4 + ((c == 0) ? (L - 1) * stride : -stride);
        stride *= L;
    }
}

// ------------------------------------------------------------------------------------------
// Wavefront-level LDS staging
// ------------------------------------------------------------------------------------------

__device__ __forceinline__ void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// 16-byte chunk as a native vector type.
typedef unsigned int chunk_t __attribute__((ext_vector_type(4)));

// Coalesced wavefront gather of spinor records through LDS, in two phases so that the global
// loads of the next gather can be in flight while the current direction computes:
//   fetch: lane l loads 16-byte chunk c = k*64 + l of the 64 records the wave needs (record
//          c / chunks, the record index of that lane obtained by a cross-lane shuffle), so
//          consecutive lanes read consecutive addresses;
//   stage: the chunks go to padded LDS slots and each lane reads its own record back.
// All 64 lanes must take part with a valid record index.

// Padded record pitch of the staging area (16-byte units; the pad spreads records over the LDS
// banks): a wavefront's area is 64 * stage_pitch<SP>() chunks.
template <class SP>
__host__ __device__ constexpr int stage_pitch() { return SP::kChunks + 1; }

template <class SP>
struct Fetch {
    chunk_t w[SP::kChunks];
    float s;
};

template <class SP>
__device__ __forceinline__ void fetch(const void *__restrict__ base, const float *__restrict__ scale, int rec,
                                      Fetch<SP> &f) {
    constexpr int CH = SP::kChunks;
    const int lane = threadIdx.x & 63;
    const chunk_t *src = reinterpret_cast<const chunk_t *>(base);
#pragma unroll
    for (int k = 0; k < CH; ++k) {
        const int c = k * 64 + lane;
        const int r = c / CH, j = c - (c / CH) * CH;
        const int n = __shfl(rec, r, 64);
        f.w[k] = src[static_cast<size_t>(n) * CH + j];
    }
    f.s = SP::kScaled ? scale[rec] : 1.0f;
}

template <class SP>
__device__ __forceinline__ void stage(const Fetch<SP> &f, chunk_t *lds, Cx<typename SP::C> p[4][3]) {
    constexpr int CH = SP::kChunks;
    constexpr int PITCH = stage_pitch<SP>();
    const int lane = threadIdx.x & 63;
#pragma unroll
    for (int k = 0; k < CH; ++k) {
        const int c = k * 64 + lane;
        const int r = c / CH, j = c - (c / CH) * CH;
        lds[r * PITCH + j] = f.w[k];
    }
    wave_sync();
    uint4 w[CH];
#pragma unroll
    for (int k = 0; k < CH; ++k) {
        const chunk_t v = lds[lane * PITCH + k];
        w[k] = make_uint4(v.x, v.y, v.z, v.w);
    }
    wave_sync();
    SP::unpack(w, f.s, p);
}

template <class SP>
__device__ __forceinline__ void gather(const void *__restrict__ base, const float *__restrict__ scale, int rec, chunk_t *lds,
                                       Cx<typename SP::C> p[4][3]) {
    Fetch<SP> f;
    fetch<SP>(base, scale, rec, f);
    stage<SP>(f, lds, p);
}

// Fifth-dimension columns inside a wavefront (the Moebius operator's fused passes): when Ls
// divides 64 and the wavefront's first lane holds s = 0, lanes lbase .. lbase + Ls - 1 hold
// s = 0 .. Ls - 1 of one 4D site, and the lanes of s + 1 and s - 1 (cyclic in the column) are
// lp and lm.
//
// stage() for the Moebius hopping pass: the lane's record becomes chi_s = b5 psi_s + c5 (S psi)_s,
// (S psi)_s = P_- psi~_{s+1} + P_+ psi~_{s-1} (P_+ the upper spins 0, 1), with cp and cm the
// factors c5 times the wall factor of s + 1 and of s - 1 (-mf across a wall, else 1).
template <class SP>
__device__ __forceinline__ void stage_b5(const Fetch<SP> &f, chunk_t *lds, Cx<typename SP::C> p[4][3], int lp, int lm,
                                         typename SP::C b5, typename SP::C cp, typename SP::C cm) {
    using C = typename SP::C;
    constexpr int CH = SP::kChunks;
    constexpr int PITCH = stage_pitch<SP>();
    const int lane = threadIdx.x & 63;
#pragma unroll
    for (int k = 0; k < CH; ++k) {
        const int c = k * 64 + lane;
        const int r = c / CH, j = c - (c / CH) * CH;
        lds[r * PITCH + j] = f.w[k];
    }
    wave_sync();
    uint4 w[CH], wp[CH], wm[CH];
#pragma unroll
    for (int k = 0; k < CH; ++k) {
        const chunk_t v = lds[lane * PITCH + k], vp = lds[lp * PITCH + k], vm = lds[lm * PITCH + k];
        w[k] = make_uint4(v.x, v.y, v.z, v.w);
        wp[k] = make_uint4(vp.x, vp.y, vp.z, vp.w);
        wm[k] = make_uint4(vm.x, vm.y, vm.z, vm.w);
    }
    wave_sync();
    float sp = f.s, sm = f.s;
    if constexpr (SP::kScaled) {
        sp = __shfl(f.s, lp, 64);
        sm = __shfl(f.s, lm, 64);
    }
    Cx<C> q[4][3];
    SP::unpack(w, f.s, p);
    SP::unpack(wm, sm, q);   // upper spins from s - 1
#pragma unroll
    for (int j = 0; j < 6; ++j) {
        Cx<C> &o = p[j / 3][j % 3];
        o = {b5 * o.r + cm * q[j / 3][j % 3].r, b5 * o.i + cm * q[j / 3][j % 3].i};
    }
    SP::unpack(wp, sp, q);   // lower spins from s + 1
#pragma unroll
    for (int j = 6; j < 12; ++j) {
        Cx<C> &o = p[j / 3][j % 3];
        o = {b5 * o.r + cp * q[j / 3][j % 3].r, b5 * o.i + cp * q[j / 3][j % 3].i};
    }
}

template <class SP>
__device__ __forceinline__ void gather_b5(const void *__restrict__ base, const float *__restrict__ scale, int rec,
                                          chunk_t *lds, Cx<typename SP::C> p[4][3], int lp, int lm, typename SP::C b5,
                                          typename SP::C cp, typename SP::C cm) {
    Fetch<SP> f;
    fetch<SP>(base, scale, rec, f);
    stage_b5<SP>(f, lds, p, lp, lm, b5, cp, cm);
}

// Half-spinor exchange inside fifth-dimension columns: h = spins 2 hf, 2 hf + 1 of lane src's v,
// through the wavefront's staging area (every lane takes part).
template <class SP>
__device__ __forceinline__ void column_half(chunk_t *lds, const Cx<typename SP::C> v[4][3], int hf, int src,
                                            Cx<typename SP::C> h[2][3]) {
    using C = typename SP::C;
    constexpr int NC = static_cast<int>(12 * sizeof(C) / 16);   // 16-byte chunks of six complex numbers
    constexpr int PITCH = stage_pitch<SP>();
    static_assert(NC <= PITCH, "a half spinor fits the lane's staging slot");
    const int lane = threadIdx.x & 63;
    C buf[12];
#pragma unroll
    for (int j = 0; j < 6; ++j) {
        buf[2 * j] = v[2 * hf + j / 3][j % 3].r;
        buf[2 * j + 1] = v[2 * hf + j / 3][j % 3].i;
    }
    chunk_t cb[NC];
    __builtin_memcpy(cb, buf, sizeof(cb));
#pragma unroll
    for (int k = 0; k < NC; ++k) lds[lane * PITCH + k] = cb[k];
    wave_sync();
#pragma unroll
    for (int k = 0; k < NC; ++k) cb[k] = lds[src * PITCH + k];
    wave_sync();
    __builtin_memcpy(buf, cb, sizeof(cb));
#pragma unroll
    for (int j = 0; j < 6; ++j) h[j / 3][j % 3] = {buf[2 * j], buf[2 * j + 1]};
}

// v = (d - S)^-1 v across a fifth-dimension column (S^dagger when dag), lanes lbase .. lbase +
// Ls - 1 holding s = 0 .. Ls - 1, r = 1 / d. S moves the lower spins from s + 1 and the upper from
// s - 1 (S^dagger the other way), with the factor -mf across the wall, so per chirality
//   x_s = sum_{j=0}^{Ls-1} c_j v_{s+-j},  c_j = r^(j+1) / (1 + mf r^Ls), times -mf once s +- j wraps,
// which is the cyclic bidiagonal system solved in closed form (stable for |d| > 1). Each half
// spinor goes through the wavefront's staging area in turn; every lane takes part.
template <class SP>
__device__ __forceinline__ void column_m5inv(chunk_t *lds, Cx<typename SP::C> v[4][3], int sl, int lbase, int Ls,
                                             typename SP::C r, typename SP::C mf, bool dag) {
    using C = typename SP::C;
    constexpr int NC = static_cast<int>(12 * sizeof(C) / 16);   // 16-byte chunks of six complex numbers
    constexpr int PITCH = stage_pitch<SP>();
    static_assert(NC <= PITCH, "a half spinor fits the lane's staging slot");
    const int lane = threadIdx.x & 63;
    C rl = C(1);
    for (int i = 0; i < Ls; ++i) rl *= r;
    const C c0 = r / (C(1) + mf * rl);
    Cx<C> x[4][3];
#pragma unroll
    for (int hf = 0; hf < 2; ++hf) {
        C buf[12];
#pragma unroll
        for (int j = 0; j < 6; ++j) {
            buf[2 * j] = v[2 * hf + j / 3][j % 3].r;
            buf[2 * j + 1] = v[2 * hf + j / 3][j % 3].i;
        }
        chunk_t cb[NC];
        __builtin_memcpy(cb, buf, sizeof(cb));
#pragma unroll
        for (int k = 0; k < NC; ++k) lds[lane * PITCH + k] = cb[k];
        wave_sync();
        const bool fwd = (hf == 1) != dag;   // this half couples to s + 1 (else to s - 1)
        Cx<C> acc[2][3];
#pragma unroll
        for (int j = 0; j < 6; ++j) acc[j / 3][j % 3] = {C(0), C(0)};
        C c = c0;
        int sj = sl;
        for (int j = 0; j < Ls; ++j) {
            if (j > 0) {
                sj += fwd ? 1 : -1;
                if (sj == Ls || sj == -1) {   // across the wall (at most once)
                    sj = fwd ? 0 : Ls - 1;
                    c *= -mf;
                }
            }
#pragma unroll
            for (int k = 0; k < NC; ++k) cb[k] = lds[(lbase + sj) * PITCH + k];
            __builtin_memcpy(buf, cb, sizeof(cb));
#pragma unroll
            for (int q = 0; q < 6; ++q) {
                Cx<C> &o = acc[q / 3][q % 3];
                o = {o.r + c * buf[2 * q], o.i + c * buf[2 * q + 1]};
            }
            c *= r;
        }
        wave_sync();
#pragma unroll
        for (int j = 0; j < 6; ++j) x[2 * hf + j / 3][j % 3] = acc[j / 3][j % 3];
    }
#pragma unroll
    for (int j = 0; j < 12; ++j) v[j / 3][j % 3] = x[j / 3][j % 3];
}

// Hardware dispatches workgroup b to XCD b % 8. Renumber so that each XCD receives one
// contiguous range of logical blocks: neighbouring lattice sites then share an L2.
__device__ __forceinline__ int xcd_block(int b, int nblocks) {
    constexpr int kXcd = 8;
    const int q = nblocks / kXcd, rem = nblocks % kXcd;
    const int xcd = b % kXcd, k = b / kXcd;
    return xcd * q + (xcd < rem ? xcd : rem) + k;
}

}  // namespace gridmi
