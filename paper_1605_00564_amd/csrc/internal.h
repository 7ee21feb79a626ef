// Internal declarations of the gfx950 solver library (not part of the ABI).
//
// Device data layout (all fields of one handle share it):
//   internal site index  idx = p*Vh + B*Vbh + j
//     p   = site parity (t+x+y+z) mod 2,
//     B   = Schwarz block, colour-major: blocks of colour 0 (Omega) first,
//           each colour in lexicographic order of the block grid,
//     j   = (local lexicographic index within the block) >> 1.
//   Block extents are even, so block origins have even parity, the local
//   parity equals the global one, and j enumerates each parity half of a
//   block exactly once.  A Schwarz block therefore owns two contiguous runs
//   of Vbh sites, one per parity, and a colour owns two contiguous halves.
//   Spinor (one right-hand side): 12 complex (spin-major, colour-minor) per
//   site, stored as chunks of 16 bytes, structure-of-arrays [chunk][V]:
//   FP64 -> 12 chunks of one complex, FP32 -> 6 chunks of two complex.
//   Multi-RHS fields are [rhs][chunk][V].
//   Links: U_mu(x) for the 4 forward directions, [mu][chunk][V]; FP64 keeps
//   all 9 entries (9 chunks of one complex), FP32 (3 chunks of 16 B) and
//   FP16/BF16 (3 chunks of 8 B) keep rows 0 and 1; row 2 = conj(row0 x row1).
//   Clover: per site two Hermitian 6x6 blocks (chirality halves, index
//   3*(spin mod 2) + colour), 36 reals each: 6 real diagonal entries, then
//   the 15 upper off-diagonal entries (i<j, row-major) as (re, im).
//   Chunks never straddle the two halves: FP64 [36][V] of double2, FP32
//   [18][V] of float4, FP16 [18][V] of 4 halfs (half h = chunks 18h/2...).
//   The inverse of the odd-site clover blocks uses the same format on the
//   odd half only ([chunk][Vh], index idx - Vh).
#pragma once
#include <hip/hip_runtime.h>
#include <hip/hip_fp16.h>
#include <hip/hip_bf16.h>

#include <cstdint>
#include <string>
#include <tuple>
#include <vector>

#include "../../include/dfl.h"

namespace dfl {

// ---------------------------------------------------------------------------
// errors
// ---------------------------------------------------------------------------
int set_error(int code, const std::string &msg);

#define DFL_HIP(call)                                                                        \
    do {                                                                                     \
        hipError_t e_ = (call);                                                              \
        if (e_ != hipSuccess)                                                                \
            return ::dfl::set_error(QCD_EHIP, std::string(#call) + ": " + hipGetErrorString(e_)); \
    } while (0)

#define DFL_TRY(call)                \
    do {                             \
        int rc_ = (call);            \
        if (rc_ < 0) return rc_;     \
    } while (0)

// ---------------------------------------------------------------------------
// complex arithmetic
// ---------------------------------------------------------------------------
// aligned to its size, so that one 8-byte (16-byte) LDS access with an
// immediate offset moves a complex float (double)
template <class R>
struct alignas(2 * sizeof(R)) cx {
    R re, im;
};

template <class R>
__host__ __device__ inline cx<R> mk(R a, R b) { return cx<R>{a, b}; }
template <class R>
__host__ __device__ inline cx<R> operator+(cx<R> a, cx<R> b) { return {a.re + b.re, a.im + b.im}; }
template <class R>
__host__ __device__ inline cx<R> operator-(cx<R> a, cx<R> b) { return {a.re - b.re, a.im - b.im}; }
template <class R>
__host__ __device__ inline cx<R> operator-(cx<R> a) { return {-a.re, -a.im}; }
template <class R>
__host__ __device__ inline cx<R> operator*(cx<R> a, cx<R> b) {
    return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re};
}
template <class R>
__host__ __device__ inline cx<R> operator*(R s, cx<R> a) { return {s * a.re, s * a.im}; }
template <class R>
__host__ __device__ inline cx<R> conj(cx<R> a) { return {a.re, -a.im}; }
// conj(a) * b
template <class R>
__host__ __device__ inline cx<R> cmulc(cx<R> a, cx<R> b) {
    return {a.re * b.re + a.im * b.im, a.re * b.im - a.im * b.re};
}
// i * a
template <class R>
__host__ __device__ inline cx<R> imul(cx<R> a) { return {-a.im, a.re}; }
template <class R>
__host__ __device__ inline R norm2(cx<R> a) { return a.re * a.re + a.im * a.im; }

// Multiply-accumulate as explicit fused multiply-adds: written as
// acc + (a b - c d) the compiler must keep a separate product and sum (it
// may not reassociate), and 0 + x cannot be folded under signed zeros, so
// sums start from their first product and continue with four FMAs per term.
__host__ __device__ inline float ffma(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
__host__ __device__ inline double ffma(double a, double b, double c) { return __builtin_fma(a, b, c); }
// acc + a b
template <class R>
__host__ __device__ inline cx<R> cmac(cx<R> acc, cx<R> a, cx<R> b) {
    return {ffma(-a.im, b.im, ffma(a.re, b.re, acc.re)), ffma(a.im, b.re, ffma(a.re, b.im, acc.im))};
}
// acc + conj(a) b
template <class R>
__host__ __device__ inline cx<R> cmacc(cx<R> acc, cx<R> a, cx<R> b) {
    return {ffma(a.im, b.im, ffma(a.re, b.re, acc.re)), ffma(-a.im, b.re, ffma(a.re, b.im, acc.im))};
}
// acc + s a (s real)
template <class R>
__host__ __device__ inline cx<R> rmac(cx<R> acc, R s, cx<R> a) {
    return {ffma(s, a.re, acc.re), ffma(s, a.im, acc.im)};
}

// ---------------------------------------------------------------------------
// storage formats
// ---------------------------------------------------------------------------
struct alignas(8) h4 { __half v[4]; };        // 2 complex in FP16
struct alignas(8) b4 { __hip_bfloat16 v[4]; }; // 2 complex in BF16
struct alignas(16) h8 { __half v[8]; };       // 4 complex in FP16
struct alignas(16) b8 { __hip_bfloat16 v[8]; }; // 4 complex in BF16

// F16R / BF16R: rows 0 and 1 in FP16 / BF16 and row 2 stored in FP32,
// computed once as conj(row0 x row1) from the rounded rows: the same matrix
// as the reconstruct-12 format, without the per-use reconstruction (for the
// ALU-bound Schwarz kernel, which reads each link many times).
enum LinkFmt { LNK_F64 = 0, LNK_F32 = 1, LNK_F16 = 2, LNK_BF16 = 3, LNK_F16R = 4, LNK_BF16R = 5 };
enum CloFmt { CLO_F64 = 0, CLO_F32 = 1, CLO_F16 = 2 };

// Device-memory tables are read and written through buffer instructions:
// the descriptor (base address) is uniform and lives in scalar registers,
// the chunk offset is a scalar offset and the site is a 32-bit per-lane
// offset, so all chunks of one site share a single VGPR address.  Every
// base handed to these helpers is within 4 GiB of the chunks it addresses
// (one right-hand side of a spinor field, one direction of the links, one
// chirality half of the clover table).
typedef unsigned u32x4_t __attribute__((ext_vector_type(4)));
typedef unsigned u32x2_t __attribute__((ext_vector_type(2)));
__device__ inline __amdgpu_buffer_rsrc_t mkrsrc(const void *p) {
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void *>(p), (short)0, (int)0xFFFFFFFFu, 0x00020000);
}
template <class T>
__device__ inline T bld(__amdgpu_buffer_rsrc_t r, unsigned soff, unsigned voff) {
    if constexpr (sizeof(T) == 16) {
        return __builtin_bit_cast(T, __builtin_amdgcn_raw_buffer_load_b128(r, (int)voff, (int)soff, 0));
    } else if constexpr (sizeof(T) == 8) {
        return __builtin_bit_cast(T, __builtin_amdgcn_raw_buffer_load_b64(r, (int)voff, (int)soff, 0));
    } else {
        static_assert(sizeof(T) == 4, "buffer element size");
        return __builtin_bit_cast(T, __builtin_amdgcn_raw_buffer_load_b32(r, (int)voff, (int)soff, 0));
    }
}
template <class T>
__device__ inline void bst(__amdgpu_buffer_rsrc_t r, unsigned soff, unsigned voff, const T &v) {
    if constexpr (sizeof(T) == 16) {
        __builtin_amdgcn_raw_buffer_store_b128(__builtin_bit_cast(u32x4_t, v), r, (int)voff, (int)soff, 0);
    } else if constexpr (sizeof(T) == 8) {
        __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u32x2_t, v), r, (int)voff, (int)soff, 0);
    } else {
        static_assert(sizeof(T) == 4, "buffer element size");
        __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned, v), r, (int)voff, (int)soff, 0);
    }
}
// element idx of chunk `chunk` of a [chunk][n] table at base
template <class T>
__device__ inline T ld(const void *base, size_t chunk, size_t n, unsigned idx) {
    return bld<T>(mkrsrc(base), (unsigned)(chunk * n * sizeof(T)), idx * (unsigned)sizeof(T));
}
// same, marked non-temporal (streamed data read once: keeps L2 for reused data)
template <class T>
__device__ inline T ld_nt(const void *base, size_t chunk, size_t n, unsigned idx) {
    const __amdgpu_buffer_rsrc_t r = mkrsrc(base);
    const unsigned soff = (unsigned)(chunk * n * sizeof(T)), voff = idx * (unsigned)sizeof(T);
    if constexpr (sizeof(T) == 16)
        return __builtin_bit_cast(T, __builtin_amdgcn_raw_buffer_load_b128(r, (int)voff, (int)soff, 2));
    else
        return __builtin_bit_cast(T, __builtin_amdgcn_raw_buffer_load_b64(r, (int)voff, (int)soff, 2));
}
template <class T>
__device__ inline void st(void *base, size_t chunk, size_t n, unsigned idx, const T &v) {
    bst<T>(mkrsrc(base), (unsigned)(chunk * n * sizeof(T)), idx * (unsigned)sizeof(T), v);
}

// Spinor storage traits.
template <class S>
struct Spin;
template <>
struct Spin<double> {
    static constexpr int NCH = 12;   // 16-byte chunks per site
    static constexpr int BYTES = 192;  // bytes per site
    template <class R>
    __device__ static inline void load(const void *base, long V, unsigned idx, cx<R> v[12]) {
#pragma unroll
        for (int k = 0; k < 12; ++k) {
            const double2 t = ld<double2>(base, k, V, idx);
            v[k] = {R(t.x), R(t.y)};
        }
    }
    template <class R>
    __device__ static inline void store(void *base, long V, unsigned idx, const cx<R> v[12]) {
#pragma unroll
        for (int k = 0; k < 12; ++k) st<double2>(base, k, V, idx, make_double2(double(v[k].re), double(v[k].im)));
    }
};
template <>
struct Spin<float> {
    static constexpr int NCH = 6;
    static constexpr int BYTES = 96;
    template <class R>
    __device__ static inline void load(const void *base, long V, unsigned idx, cx<R> v[12]) {
#pragma unroll
        for (int c = 0; c < 6; ++c) {
            const float4 t = ld<float4>(base, c, V, idx);
            v[2 * c] = {R(t.x), R(t.y)};
            v[2 * c + 1] = {R(t.z), R(t.w)};
        }
    }
    template <class R>
    __device__ static inline void store(void *base, long V, unsigned idx, const cx<R> v[12]) {
#pragma unroll
        for (int c = 0; c < 6; ++c)
            st<float4>(base, c, V, idx,
                       make_float4(float(v[2 * c].re), float(v[2 * c].im), float(v[2 * c + 1].re),
                                   float(v[2 * c + 1].im)));
    }
};

// The power-of-two scale of an FP16 vector whose largest |re| or |im| is m:
// m = f 2^e with f in [0.5, 1) (e = biased exponent - 126); the scale 2^(e-15)
// and its inverse are built from exponent bits, and vectors whose largest
// entry is below 2^-112 are stored as zero.
__device__ inline void r16_scale(float m, float &sc, float &inv) {
    const int eb = (int)((__float_as_uint(m) >> 23) & 0xffu);
    const bool nz = eb >= 15;
    sc = nz ? __uint_as_float((unsigned)(eb - 14) << 23) : 0.f;
    inv = nz ? __uint_as_float((unsigned)(268 - eb) << 23) : 0.f;
}

// FP16 spinor with a per-site power-of-two scale: a right-hand side holds
// 3 chunks of [V] x 8 halves (4 complex each), then [V] FP32 scales (52 V
// bytes).  The scale 2^e puts the site's largest |re| or |im| in
// [2^14, 2^15) before rounding, so every site keeps FP16's full relative
// precision whatever the field's dynamic range, and the scaling is exact.
template <>
struct Spin<__half> {
    static constexpr int NCH = 3;
    static constexpr int BYTES = 52;
    template <class R>
    __device__ static inline void decode(const h8 t[3], float sc, cx<R> v[12]) {
#pragma unroll
        for (int c = 0; c < 3; ++c)
#pragma unroll
            for (int e = 0; e < 4; ++e)
                v[4 * c + e] = {R(__half2float(t[c].v[2 * e]) * sc), R(__half2float(t[c].v[2 * e + 1]) * sc)};
    }
    template <class R>
    __device__ static inline void load(const void *base, long V, unsigned idx, cx<R> v[12]) {
        h8 t[3];
#pragma unroll
        for (int c = 0; c < 3; ++c) t[c] = ld<h8>(base, c, V, idx);
        decode(t, ld<float>(base, 12, V, idx), v);
    }
    template <class R>
    __device__ static inline void encode(const cx<R> v[12], h8 t[3], float &sc) {
        float m = 0.f;
#pragma unroll
        for (int k = 0; k < 12; ++k) m = fmaxf(m, fmaxf(fabsf(float(v[k].re)), fabsf(float(v[k].im))));
        float inv;
        r16_scale(m, sc, inv);
#pragma unroll
        for (int c = 0; c < 3; ++c)
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                t[c].v[2 * q] = __float2half_rn(float(v[4 * c + q].re) * inv);
                t[c].v[2 * q + 1] = __float2half_rn(float(v[4 * c + q].im) * inv);
            }
    }
    template <class R>
    __device__ static inline void store(void *base, long V, unsigned idx, const cx<R> v[12]) {
        h8 t[3];
        float sc;
        encode(v, t, sc);
#pragma unroll
        for (int c = 0; c < 3; ++c) st<h8>(base, c, V, idx, t[c]);
        st<float>(base, 12, V, idx, sc);
    }
};

// bytes of one spinor (one RHS) in each storage type (F16 = FP16 with scale)
inline size_t spinor_bytes(qcd_prec p, long V) {
    return (p == QCD_F64 ? 192 : p == QCD_F16 ? 52 : 96) * (size_t)V;
}

// Link access: 3x3 matrix W of site idx and direction mu.
template <int F>
struct Link;
template <>
struct Link<LNK_F64> {
    template <class R>
    __device__ static inline void load(const void *base, long V, int mu, unsigned idx, cx<R> w[9]) {
#pragma unroll
        for (int k = 0; k < 9; ++k) {
            const double2 t = ld<double2>(static_cast<const double2 *>(base) + (size_t)mu * 9 * V, k, V, idx);
            w[k] = {R(t.x), R(t.y)};
        }
    }
};
template <class R>
__device__ inline void rebuild_row2(cx<R> w[9]) {
    // row2 = conj(row0 x row1)
    w[6] = conj(cmac(w[1] * w[5], -w[2], w[4]));
    w[7] = conj(cmac(w[2] * w[3], -w[0], w[5]));
    w[8] = conj(cmac(w[0] * w[4], -w[1], w[3]));
}
template <>
struct Link<LNK_F32> {
    template <class R>
    __device__ static inline void load(const void *base, long V, int mu, unsigned idx, cx<R> w[9]) {
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            const float4 t = ld<float4>(static_cast<const float4 *>(base) + (size_t)mu * 3 * V, c, V, idx);
            w[2 * c] = {R(t.x), R(t.y)};
            w[2 * c + 1] = {R(t.z), R(t.w)};
        }
        rebuild_row2(w);
    }
};
template <>
struct Link<LNK_F16> {
    template <class R>
    __device__ static inline void load(const void *base, long V, int mu, unsigned idx, cx<R> w[9]) {
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            const h4 t = ld<h4>(static_cast<const h4 *>(base) + (size_t)mu * 3 * V, c, V, idx);
            w[2 * c] = {R(__half2float(t.v[0])), R(__half2float(t.v[1]))};
            w[2 * c + 1] = {R(__half2float(t.v[2])), R(__half2float(t.v[3]))};
        }
        rebuild_row2(w);
    }
};
template <>
struct Link<LNK_BF16> {
    template <class R>
    __device__ static inline void load(const void *base, long V, int mu, unsigned idx, cx<R> w[9]) {
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            const b4 t = ld<b4>(static_cast<const b4 *>(base) + (size_t)mu * 3 * V, c, V, idx);
            w[2 * c] = {R(__bfloat162float(t.v[0])), R(__bfloat162float(t.v[1]))};
            w[2 * c + 1] = {R(__bfloat162float(t.v[2])), R(__bfloat162float(t.v[3]))};
        }
        rebuild_row2(w);
    }
};

// [mu][3 chunks of 16 B][V]: chunk 0 = w0..w3 in the half type, chunk 1 =
// w4, w5 (half type) and w6 (FP32), chunk 2 = w7, w8 (FP32)
__device__ inline float to_f(__half x) { return __half2float(x); }
__device__ inline float to_f(__hip_bfloat16 x) { return __bfloat162float(x); }
template <class H4, class H8>
struct LinkR {
    template <class R>
    __device__ static inline void load(const void *base, long V, int mu, unsigned idx, cx<R> w[9]) {
        const float4 *b = static_cast<const float4 *>(base) + (size_t)mu * 3 * V;
        const H8 t0 = ld<H8>(b, 0, V, idx);
        const float4 t1 = ld<float4>(b, 1, V, idx);
        const float4 t2 = ld<float4>(b, 2, V, idx);
        H4 t1h;
        __builtin_memcpy(&t1h, &t1, sizeof(H4));
#pragma unroll
        for (int k = 0; k < 4; ++k) w[k] = {R(to_f(t0.v[2 * k])), R(to_f(t0.v[2 * k + 1]))};
        w[4] = {R(to_f(t1h.v[0])), R(to_f(t1h.v[1]))};
        w[5] = {R(to_f(t1h.v[2])), R(to_f(t1h.v[3]))};
        w[6] = {R(t1.z), R(t1.w)};
        w[7] = {R(t2.x), R(t2.y)};
        w[8] = {R(t2.z), R(t2.w)};
    }
};
template <>
struct Link<LNK_F16R> : LinkR<h4, h8> {};
template <>
struct Link<LNK_BF16R> : LinkR<b4, b8> {};

// Clover access: one chirality half (36 reals) of a site's packed clover;
// NT marks the loads non-temporal (clover read once per site by the stencil).
template <class T, bool NT>
__device__ inline T ldc(const void *base, size_t chunk, size_t n, unsigned idx) {
    if constexpr (NT)
        return ld_nt<T>(base, chunk, n, idx);
    else
        return ld<T>(base, chunk, n, idx);
}
template <int F>
struct Clo;
template <>
struct Clo<CLO_F64> {
    template <class R, bool NT = false>
    __device__ static inline void load_half(const void *base, long n, unsigned at, int h, R a[36]) {
#pragma unroll
        for (int k = 0; k < 18; ++k) {
            const double2 t = ldc<double2, NT>(static_cast<const double2 *>(base) + (size_t)h * 18 * n, k, n, at);
            a[2 * k] = R(t.x);
            a[2 * k + 1] = R(t.y);
        }
    }
};
template <>
struct Clo<CLO_F32> {
    template <class R, bool NT = false>
    __device__ static inline void load_half(const void *base, long n, unsigned at, int h, R a[36]) {
#pragma unroll
        for (int k = 0; k < 9; ++k) {
            const float4 t = ldc<float4, NT>(static_cast<const float4 *>(base) + (size_t)h * 9 * n, k, n, at);
            a[4 * k] = R(t.x);
            a[4 * k + 1] = R(t.y);
            a[4 * k + 2] = R(t.z);
            a[4 * k + 3] = R(t.w);
        }
    }
};
template <>
struct Clo<CLO_F16> {
    template <class R, bool NT = false>
    __device__ static inline void load_half(const void *base, long n, unsigned at, int h, R a[36]) {
#pragma unroll
        for (int k = 0; k < 9; ++k) {
            const h4 t = ldc<h4, NT>(static_cast<const h4 *>(base) + (size_t)h * 9 * n, k, n, at);
#pragma unroll
            for (int e = 0; e < 4; ++e) a[4 * k + e] = R(__half2float(t.v[e]));
        }
    }
};

// out = H v for one packed Hermitian 6x6 block h (36 reals) and 6-vector v.
template <class R>
__device__ inline void herm6_apply(const R *h, const cx<R> v[6], cx<R> out[6]) {
#pragma unroll
    for (int i = 0; i < 6; ++i) out[i] = h[i] * v[i];
    int m = 0;
#pragma unroll
    for (int i = 0; i < 6; ++i)
#pragma unroll
        for (int j = i + 1; j < 6; ++j) {
            cx<R> a = {h[6 + 2 * m], h[7 + 2 * m]};
            out[i] = cmac(out[i], a, v[j]);
            out[j] = cmacc(out[j], a, v[i]);
            ++m;
        }
}

// out = A v for the clover of site `at` of a table with n entries, read and
// applied one chirality half at a time.
template <int CF, class R, bool NT = false>
__device__ inline void clover_apply(const void *clo, long n, unsigned at, const cx<R> v[12], cx<R> out[12]) {
#pragma unroll
    for (int h = 0; h < 2; ++h) {
        R a[36];
        Clo<CF>::template load_half<R, NT>(clo, n, at, h, a);
        herm6_apply(a, v + 6 * h, out + 6 * h);
    }
}

// ---------------------------------------------------------------------------
// hopping term pieces: (1 + s gamma_mu) W psi accumulated into acc, with the
// chiral-basis spin projection (two colour vectors h0, h1 carry the result).
// ---------------------------------------------------------------------------
template <class R, int MU, int S>
__device__ inline void project(const cx<R> p[12], cx<R> h[6]) {
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        const cx<R> p0 = p[c], p1 = p[3 + c], p2 = p[6 + c], p3 = p[9 + c];
        if (MU == 0) {
            h[c] = S > 0 ? p0 - p2 : p0 + p2;
            h[3 + c] = S > 0 ? p1 - p3 : p1 + p3;
        } else if (MU == 1) {
            h[c] = S > 0 ? p0 - imul(p3) : p0 + imul(p3);
            h[3 + c] = S > 0 ? p1 - imul(p2) : p1 + imul(p2);
        } else if (MU == 2) {
            h[c] = S > 0 ? p0 - p3 : p0 + p3;
            h[3 + c] = S > 0 ? p1 + p2 : p1 - p2;
        } else {
            h[c] = S > 0 ? p0 - imul(p2) : p0 + imul(p2);
            h[3 + c] = S > 0 ? p1 + imul(p3) : p1 - imul(p3);
        }
    }
}

// acc + s i a (s real)
template <class R>
__device__ inline cx<R> imac(cx<R> acc, R s, cx<R> a) {
    return {ffma(-s, a.im, acc.re), ffma(s, a.re, acc.im)};
}

template <class R, int MU, int S>
__device__ inline void reconstruct_add(const cx<R> g[6], R sign, cx<R> acc[12]) {
    // the hop's boundary sign enters through the FMAs (a constant 1 folds away)
    const R sp = S > 0 ? sign : -sign, sm = -sp;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        const cx<R> g0 = g[c], g1 = g[3 + c];
        acc[c] = rmac(acc[c], sign, g0);
        acc[3 + c] = rmac(acc[3 + c], sign, g1);
        if (MU == 0) {  // (h0, h1, -s h0, -s h1)
            acc[6 + c] = rmac(acc[6 + c], sm, g0);
            acc[9 + c] = rmac(acc[9 + c], sm, g1);
        } else if (MU == 1) {  // (h0, h1, i s h1, i s h0)
            acc[6 + c] = imac(acc[6 + c], sp, g1);
            acc[9 + c] = imac(acc[9 + c], sp, g0);
        } else if (MU == 2) {  // (h0, h1, s h1, -s h0)
            acc[6 + c] = rmac(acc[6 + c], sp, g1);
            acc[9 + c] = rmac(acc[9 + c], sm, g0);
        } else {  // (h0, h1, i s h0, -i s h1)
            acc[6 + c] = imac(acc[6 + c], sp, g0);
            acc[9 + c] = imac(acc[9 + c], sm, g1);
        }
    }
}

// g = W h (DAG=false) or W^+ h (DAG=true) on both colour vectors of h.
template <class R, bool DAG>
__device__ inline void su3_mul2(const cx<R> w[9], const cx<R> h[6], cx<R> g[6]) {
#pragma unroll
    for (int s = 0; s < 2; ++s)
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            cx<R> acc = DAG ? cmulc(w[a], h[3 * s]) : w[a * 3] * h[3 * s];
#pragma unroll
            for (int b = 1; b < 3; ++b)
                acc = DAG ? cmacc(acc, w[b * 3 + a], h[3 * s + b]) : cmac(acc, w[a * 3 + b], h[3 * s + b]);
            g[3 * s + a] = acc;
        }
}

// acc += sign * (1 - gamma_mu) U psi   (forward hop)  or
// acc += sign * (1 + gamma_mu) U^+ psi (backward hop)
template <class R, int MU, bool FWD>
__device__ inline void hop(const cx<R> w[9], const cx<R> psi[12], R sign, cx<R> acc[12]) {
    constexpr int S = FWD ? -1 : +1;
    cx<R> h[6], g[6];
    project<R, MU, S>(psi, h);
    su3_mul2<R, !FWD>(w, h, g);
    reconstruct_add<R, MU, S>(g, sign, acc);
}

// SplitMix64 (Steele, Lea, Flood 2014) as a counter-based generator: output
// n of the sequence started at state `key`
__host__ __device__ inline unsigned long long sm64(unsigned long long key, unsigned long long n) {
    unsigned long long z = key + (n + 1ULL) * 0x9E3779B97F4A7C15ULL;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    return z ^ (z >> 31);
}

// A pointer the caller knows to be the same in every lane, marked as such:
// buffer loads need their descriptor in scalar registers, and where the
// compiler cannot prove a base uniform it wraps each load in a loop over
// the distinct values.
template <class T>
__device__ inline T *wave_uniform(T *p) {
    const unsigned long long v = reinterpret_cast<unsigned long long>(p);
    const unsigned lo = __builtin_amdgcn_readfirstlane((unsigned)v);
    const unsigned hi = __builtin_amdgcn_readfirstlane((unsigned)(v >> 32));
    return reinterpret_cast<T *>(((unsigned long long)hi << 32) | lo);
}

// XCD-aware order of a 2D grid.  Workgroups are dispatched round-robin over
// the 8 XCDs (each with its own L2) by linear id; this maps them so that XCD k
// gets the k-th contiguous eighth of the logical grid, with all y (right-hand
// side groups) of one x (site tile or Schwarz block) adjacent, so that link,
// clover and neighbour data are reused inside one L2.
__device__ inline void xcd_order(unsigned &x, unsigned &y) {
    const unsigned gx = gridDim.x, gy = gridDim.y, tot = gx * gy;
    if (tot % 8u) {
        x = blockIdx.x;
        y = blockIdx.y;
        return;
    }
    const unsigned w = blockIdx.x + blockIdx.y * gx;
    const unsigned L = (w & 7u) * (tot >> 3) + (w >> 3);
    x = L / gy;
    y = L - x * gy;
}

// neighbour table: entry of site x in direction d = 2 mu + (0 fwd | 1 bwd);
// bit 31 marks the antiperiodic time-boundary sign
__device__ inline int nbr_at(const int *nbr, int d, long V, unsigned x) { return ld<int>(nbr, d, V, x); }
__device__ inline unsigned nb_index(int e) { return (unsigned)(e & 0x7fffffff); }
template <class R>
__device__ inline R nb_sign(int e) { return e < 0 ? R(-1) : R(1); }

// ---------------------------------------------------------------------------
// geometry and the field handle
// ---------------------------------------------------------------------------
// Largest byte offset per lattice site that one buffer access adds to a
// table base (chunk offset + element offset); make_geom rejects lattices
// for which it reaches 2^32.
constexpr unsigned long long MAX_OFFSET_BYTES_PER_SITE = 384;

struct Geom {
    int L[4], b[4], nb[4];
    long V, Vh;
    int Vb, Vbh, Nb;
};

}  // namespace dfl

struct qcd_field_s {
    qcd_lattice lat;
    dfl::Geom g;
    int device = 0;
    int *nbr = nullptr;      // [8][V], direction d = 2*mu + (0 fwd | 1 bwd)
    short *lnbr = nullptr;   // [2 parity][Vbh][8]: in-block neighbour (local j) or -1; same for every block
    // hops leaving a block, per direction mu: entries (parity << 30 | fwd 0 / bwd 1 << 29 | j),
    // [4][face_cap], nface[mu] used; the same for every block
    int *bface = nullptr;
    int nface[4] = {0, 0, 0, 0};
    int face_cap = 0;
    // per entry of bface: the site across the face, in the neighbouring
    // block, that feeds it (parity << 30 | j); [4][face_cap]
    int *bfsrc = nullptr;
    // [Nb][8], block B (memory order) and entry kind 2 mu + d (d of bface):
    // the block whose face entries of that kind B feeds (B - mu for d = 0,
    // B + mu for d = 1), in memory order; bit 31: the hop crosses the
    // antiperiodic time boundary
    int *bfnb = nullptr;
    int nface_tot = 0;       // sum of nface: face entries per block
    int *int_of = nullptr;   // [V] lexicographic -> internal
    int *lex_of = nullptr;   // [V] internal -> lexicographic
    int *border = nullptr;   // [Nb] lexicographic block -> block index in memory (colour-major)
    void *U[6] = {nullptr, nullptr, nullptr, nullptr, nullptr, nullptr};  // by LinkFmt
    void *clo[3] = {nullptr, nullptr, nullptr};             // by CloFmt, all sites
    void *cloinv[3] = {nullptr, nullptr, nullptr};          // by CloFmt, odd sites
    void *Uape = nullptr;    // APE-smeared spatial links, FP64 [3][9][V] (smearing of sources and sinks)
    // scratch buffers owned by the handle, one per purpose, grown on demand
    void *buf[11] = {nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr};
    size_t buf_bytes[11] = {0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0};
    int *flag = nullptr;     // device status word
    unsigned graph_gen = 0;  // bumped whenever a scratch buffer moves (captured graphs refer to them)
    // stencil launch choices (autotuner knobs; defaults from the environment)
    int st_block = 1;        // block-staged kernel when the block fits (0: site tiles)
    int st_rg = 0;           // right-hand sides per site tile (0: automatic)
    int st_order = 1;        // site tiles in lexicographic block order (0: memory order)
    int st_nr = 0;           // block-staged kernel: right-hand sides per workgroup (0: automatic)
    int st_linklds = 1;      // FP32 vectors, half links, >= 16 rhs: links in LDS, rhs looped
    int st_sap_pair = 1;     // Schwarz sweep: two right-hand sides per workgroup (4^4 blocks)
    size_t lds_max = 64 * 1024;   // the device's LDS bytes per workgroup
    void *graphs = nullptr;  // captured solve graphs (owned; see batched.hip)
    hipStream_t cap = nullptr;  // library stream used for stream capture
    double *hp = nullptr;    // pinned host scratch (4096 doubles)
};

namespace dfl {

// grow-only device scratch of a field handle, one buffer per purpose
enum BufSlot {
    BUF_APPLY = 0, BUF_SAP = 1, BUF_GCR = 2, BUF_GCR_IO = 3, BUF_DFL = 4, BUF_AMA = 5, BUF_RED = 6, BUF_SAP_IO = 7,
    BUF_RES = 8, BUF_CONTRACT = 9, BUF_SAP_RES = 10
};
int field_buffer(qcd_field f, int slot, size_t bytes, void **p);
// Solver mode without host synchronisation (for stream capture into a HIP
// graph): no host reads of norms, fixed iteration counts, little solves with
// a fixed budget, no profiling events.  Per host thread.
void set_nosync(bool on);
bool nosync();
// set while a solve is being captured: workspace must not grow (a captured
// graph keeps the addresses it saw)
void set_capturing(bool on);
bool capturing();
// captured graphs of a field handle (batched solves); freed with the handle
void graph_cache_free(qcd_field f);
// process-wide cache of call-scoped device workspace, per device
int ws_acquire(int dev, size_t bytes, void **p, size_t *got);
void ws_release(int dev, void *p, size_t bytes);
size_t ws_cached_bytes(int dev);   // held in the cache, available to new requests
bool dev_alloc(int dev, void **p, size_t bytes);   // hipMalloc, freeing the cache on failure

// Profiling of kernel classes with HIP events.
enum ProfClass { PROF_DIRAC = 0, PROF_SAP = 1, PROF_DFL = 2, PROF_LITTLE = 3, PROF_BLAS = 4, PROF_OTHER = 5 };
// One scope per kernel launch of a class: HIP events on the launch stream
// bracket it, and the launch's algorithmic work (flops, compulsory HBM bytes,
// work units: site-applications per right-hand side) is accumulated.
struct ProfScope {
    int cls;
    hipStream_t s;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    ProfScope(int cls, hipStream_t s, double flops = 0, double bytes = 0, double units = 0);
    ~ProfScope();
};

// link / clover storage chosen for a precision request
inline LinkFmt link_fmt(qcd_prec p) {
    return p == QCD_F64 ? LNK_F64 : p == QCD_F32 ? LNK_F32 : p == QCD_F16 ? LNK_F16 : LNK_BF16;
}
inline CloFmt clo_fmt(qcd_prec p) { return p == QCD_F64 ? CLO_F64 : p == QCD_F32 ? CLO_F32 : CLO_F16; }

// --- internal operations (device pointers in the internal layout) ---------
// out = M in on internal vectors; nrhs fields of type S (double or float)
// r = b - M x with the FP64 operator and ||r||^2 per right-hand side into
// `norm2` (device, n doubles); internal FP64 vectors.  rho32 (optional):
// also r rounded to internal FP32 vectors
int dirac_resid(qcd_field f, const double2 *x, const double2 *b, double2 *r, int nrhs, double *norm2,
                hipStream_t s, float4 *rho32 = nullptr);
int dirac_internal2(qcd_field f, const void *in, qcd_prec vin, void *out, qcd_prec vout, int nrhs,
                    qcd_prec storage, hipStream_t s);
int dirac_internal(qcd_field f, const void *in, void *out, int nrhs, qcd_prec vec, qcd_prec storage,
                   hipStream_t s);
// psi = M_SAP eta on internal vectors (FP32 vectors unless sap.storage == F64)
int sap_internal(qcd_field f, const qcd_sap *sap, const void *eta, void *psi, int nrhs, hipStream_t s);
// GCR on FP64 internal vectors b -> x (info: host array of n, may be null)
int gcr_internal(qcd_field f, const qcd_gcr *p, const double2 *b, double2 *x, int n, qcd_info *info,
                 hipStream_t s);
// n right-hand sides b64 -> x64 (internal FP64), eagerly with the
// residual-stopping solver (graph = false) or, for a fixed iteration count,
// replayed from a HIP graph captured on the first call with this batch size,
// parameters and workspace vectors; status becomes QCD_NOCONV if any
// solution misses p.res
// right-hand sides per solver launch for parameters p: want (> 0), lowered
// to an even count only if 90% of the available memory cannot hold it, or
// (want = 0) what 60% of it holds, at most 48 and a multiple of 12 when
// possible; available: free memory, the workspace cache and the handle's
// buffers other than slot `busy`
int pick_batch(qcd_field f, const qcd_gcr &p, int want, int busy = -1);
int solve_batch(qcd_field f, const qcd_gcr &p, const double2 *b64, double2 *x64, int n, bool graph, qcd_info *info,
                hipStream_t s, int &status);
// canonical <-> internal conversion; canon is complex128 (F64) or complex64 (F32)
int pack_spinor(qcd_field f, const void *canon, qcd_prec io, void *internal, qcd_prec vec, int nrhs,
                hipStream_t s);
int unpack_spinor(qcd_field f, const void *internal, qcd_prec vec, void *canon, qcd_prec io, int nrhs,
                  hipStream_t s);

// one source vector built in the internal FP64 layout: Z2 noise vector
// `index` of the stream `seed`; the sequential source of one canonical
// forward solution (io precision) on timeslice t_sink with the
// gamma_5 gamma_mu gamma_5 insertion
int z2_source_internal(qcd_field f, unsigned long long seed, long long index, double2 *b, hipStream_t s);
int seq_source_internal(qcd_field f, const void *fwd, qcd_prec io, int t_sink, int mu, double2 *b, hipStream_t s);

// device address of the static scratch array of dirac_apply_noalloc,
// looked up once per device with that device current (at field creation)
int static_scratch_init(int dev);

// launch geometry helper: grid of g workgroups over n items
inline unsigned nblocks(long n, int bs) { return (unsigned)((n + bs - 1) / bs); }

}  // namespace dfl
