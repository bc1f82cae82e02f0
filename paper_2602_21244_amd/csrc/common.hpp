// Shared device/host helpers of the gfx950 DSMC library.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/dsmc.h"

namespace dsmc {

// --------------------------------------------------------------------------
// Error reporting (host)
// --------------------------------------------------------------------------
void set_error(const char* fmt, ...);
int arg_error(const char* fmt, ...);
int hip_check(hipError_t e, const char* what);

#define DSMC_LAUNCH_CHECK(what)                                                   \
    do {                                                                          \
        hipError_t e_ = hipGetLastError();                                        \
        if (e_ != hipSuccess) return ::dsmc::hip_check(e_, what);                 \
    } while (0)

// Persistent grid for data-dependent sizes (pair counts live on the device).
int persistent_blocks(int threads_per_block);
dsmc_match_schedule match_schedule();
// Compute units of the current device.
int device_cus();

inline hipStream_t as_stream(dsmc_stream_t s) { return reinterpret_cast<hipStream_t>(s); }

inline size_t align_up(size_t x, size_t a = 256) { return (x + a - 1) / a * a; }

// --------------------------------------------------------------------------
// Counter-based RNG: Philox4x32-10 (Salmon et al., SC'11), counter
// (c0, cell, step, slot), key = seed.
// --------------------------------------------------------------------------
struct U4 { uint32_t a, b, c, d; };

__device__ __forceinline__ U4 philox10(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3,
                                       uint32_t k0, uint32_t k1)
{
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        // one 32 x 32 -> 64-bit product gives both halves (v_mad_u64_u32)
        const uint64_t p0 = (uint64_t)0xD2511F53u * c0;
        const uint64_t p1 = (uint64_t)0xCD9E8D57u * c2;
        const uint32_t n0 = (uint32_t)(p1 >> 32) ^ c1 ^ k0;
        const uint32_t n2 = (uint32_t)(p0 >> 32) ^ c3 ^ k1;
        c0 = n0; c1 = (uint32_t)p1; c2 = n2; c3 = (uint32_t)p0;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    return U4{c0, c1, c2, c3};
}

enum : uint32_t { SLOT_CAND = 0, SLOT_COUNT = 1, SLOT_LAT0 = 2, SLOT_LAT1 = 3, SLOT_LAT2 = 4,
                  SLOT_SBT = 5 };

__device__ __forceinline__ U4 draw(const dsmc_rng& rng, uint32_t c0, uint32_t cell, uint32_t slot)
{
    return philox10(c0, cell, rng.step, slot, (uint32_t)rng.seed, (uint32_t)(rng.seed >> 32));
}

// [0,1) with 53 random bits from two words.
__device__ __forceinline__ double unif53(uint32_t a, uint32_t b)
{
    return ((double)(a >> 5) * 67108864.0 + (double)(b >> 6)) * 0x1.0p-53;
}
// [0,1) with 24 random bits.
__device__ __forceinline__ float unif24(uint32_t a) { return (float)(a >> 8) * 0x1.0p-24f; }

// Uniforms of one accepted pair (index a in its cell), in two groups:
// U[0..3] feed xi (slot 2, and slot 3 for 53-bit uniforms), U[4..5] feed z
// (slot 4 for 53-bit uniforms, slot 3 for 24-bit ones).
__device__ __forceinline__ void uniforms_xi(const dsmc_rng& rng, uint32_t a, uint32_t cell,
                                            double (&U)[4])
{
    const U4 r0 = draw(rng, a, cell, SLOT_LAT0);
    const U4 r1 = draw(rng, a, cell, SLOT_LAT1);
    U[0] = unif53(r0.a, r0.b); U[1] = unif53(r0.c, r0.d);
    U[2] = unif53(r1.a, r1.b); U[3] = unif53(r1.c, r1.d);
}
__device__ __forceinline__ void uniforms_z(const dsmc_rng& rng, uint32_t a, uint32_t cell,
                                           double (&U)[2])
{
    const U4 r2 = draw(rng, a, cell, SLOT_LAT2);
    U[0] = unif53(r2.a, r2.b); U[1] = unif53(r2.c, r2.d);
}
__device__ __forceinline__ void uniforms_xi(const dsmc_rng& rng, uint32_t a, uint32_t cell,
                                            float (&U)[4])
{
    const U4 r0 = draw(rng, a, cell, SLOT_LAT0);
    U[0] = unif24(r0.a); U[1] = unif24(r0.b); U[2] = unif24(r0.c); U[3] = unif24(r0.d);
}
__device__ __forceinline__ void uniforms_z(const dsmc_rng& rng, uint32_t a, uint32_t cell,
                                           float (&U)[2])
{
    const U4 r1 = draw(rng, a, cell, SLOT_LAT1);
    U[0] = unif24(r1.a); U[1] = unif24(r1.b);
}

// Box-Muller (Box & Muller 1958); 1-U keeps the log argument in (0, 1].
__device__ __forceinline__ void box_muller(double ua, double ub, double& n1, double& n2)
{
    const double R = sqrt(-2.0 * log(1.0 - ua));
    double s, c;
    sincospi(2.0 * ub, &s, &c);
    n1 = R * c;
    n2 = R * s;
}
__device__ __forceinline__ void box_muller(float ua, float ub, float& n1, float& n2)
{
    const float R = sqrtf(-2.0f * logf(1.0f - ua));
    float s, c;
    sincospif(2.0f * ub, &s, &c);
    n1 = R * c;
    n2 = R * s;
}

// Latents of a pair: xi (3) and z (2) normals, plus U[4] (= b^2 / b_max^2).
// The two halves are separate so that two lanes can share one pair's work.
template <typename T>
__device__ __forceinline__ void latents_xi(const dsmc_rng& rng, uint32_t a, uint32_t cell,
                                           T (&xi)[3])
{
    T U[4];
    uniforms_xi(rng, a, cell, U);
    T spare;
    box_muller(U[0], U[1], xi[0], xi[1]);
    box_muller(U[2], U[3], xi[2], spare);
}
template <typename T>
__device__ __forceinline__ void latents_z(const dsmc_rng& rng, uint32_t a, uint32_t cell,
                                          T (&z)[2], T& u4)
{
    T U[2];
    uniforms_z(rng, a, cell, U);
    box_muller(U[0], U[1], z[0], z[1]);
    u4 = U[0];
}
template <typename T>
__device__ __forceinline__ void pair_latents(const dsmc_rng& rng, uint32_t a, uint32_t cell,
                                             T (&xi)[3], T (&z)[2], T& u4)
{
    latents_xi(rng, a, cell, xi);
    latents_z(rng, a, cell, z, u4);
}

// --------------------------------------------------------------------------
// Small vector helpers
// --------------------------------------------------------------------------
template <typename T> __device__ __forceinline__ T dev_sqrt(T x);
template <> __device__ __forceinline__ double dev_sqrt<double>(double x) { return sqrt(x); }
template <> __device__ __forceinline__ float dev_sqrt<float>(float x) { return sqrtf(x); }

// Unit vector of (a,b,c) (x axis if zero); returns the norm.
template <typename T>
__device__ __forceinline__ T unit3(T a, T b, T c, T (&o)[3])
{
    const T n = dev_sqrt<T>(a * a + b * b + c * c);
    if (n > T(0)) {
        const T inv = T(1) / n;
        o[0] = a * inv; o[1] = b * inv; o[2] = c * inv;
    } else {
        o[0] = T(1); o[1] = T(0); o[2] = T(0);
    }
    return n;
}

// Unit vector along the part of xi orthogonal to vh (vh unit).
template <typename T>
__device__ __forceinline__ void perp_dir(const T (&xi)[3], const T (&vh)[3], T (&e)[3])
{
    const T d = xi[0] * vh[0] + xi[1] * vh[1] + xi[2] * vh[2];
    T w0 = xi[0] - d * vh[0], w1 = xi[1] - d * vh[1], w2 = xi[2] - d * vh[2];
    T n = dev_sqrt<T>(w0 * w0 + w1 * w1 + w2 * w2);
    if (!(n > T(0))) {
        // xi parallel to vh: cross product with the axis of vh's smallest component
        const T ax = fabs(vh[0]), ay = fabs(vh[1]), az = fabs(vh[2]);
        T t0 = 0, t1 = 0, t2 = 0;
        if (ax <= ay && ax <= az) t0 = 1; else if (ay <= az) t1 = 1; else t2 = 1;
        w0 = vh[1] * t2 - vh[2] * t1;
        w1 = vh[2] * t0 - vh[0] * t2;
        w2 = vh[0] * t1 - vh[1] * t0;
        n = dev_sqrt<T>(w0 * w0 + w1 * w1 + w2 * w2);
    }
    const T inv = T(1) / n;
    e[0] = w0 * inv; e[1] = w1 * inv; e[2] = w2 * inv;
}

// Status word updates (device).
__device__ __forceinline__ void st_flag(dsmc_status* st, uint32_t f)
{
    if (st) atomicOr(&st->flags, f);
}

// Wave64 reductions with cross-lane shuffles.
// Value of the partner lane under a DPP pattern inside each 16-lane row
// (quad_perm [1,0,3,2], quad_perm [2,3,0,1], row_half_mirror, row_mirror):
// a VALU move instead of an LDS-crossbar permute.  Needs the whole wave
// active, as every wave reduction here is called.
template <int CTRL>
__device__ __forceinline__ double dpp_partner(double x)
{
    const uint64_t b = __builtin_bit_cast(uint64_t, x);
    const int l0 = (int)(uint32_t)b, h0 = (int)(uint32_t)(b >> 32);
    const int lo = __builtin_amdgcn_update_dpp(l0, l0, CTRL, 0xF, 0xF, false);
    const int hi = __builtin_amdgcn_update_dpp(h0, h0, CTRL, 0xF, 0xF, false);
    return __builtin_bit_cast(double, ((uint64_t)(uint32_t)hi << 32) | (uint32_t)lo);
}
constexpr int DPP_QUAD_XOR1 = 0xB1, DPP_QUAD_XOR2 = 0x4E, DPP_ROW_HALF_MIRROR = 0x141,
              DPP_ROW_MIRROR = 0x140;

// Butterfly sum over the wave: pairs within quads, then quads and half-rows
// by mirrors, then rows by lane shuffles.  Every pairing is symmetric, so
// all lanes end with the same bits, and the order is fixed.
__device__ __forceinline__ double wave_sum(double x)
{
    x += dpp_partner<DPP_QUAD_XOR1>(x);
    x += dpp_partner<DPP_QUAD_XOR2>(x);
    x += dpp_partner<DPP_ROW_HALF_MIRROR>(x);
    x += dpp_partner<DPP_ROW_MIRROR>(x);
    x += __shfl_xor(x, 16, 64);
    x += __shfl_xor(x, 32, 64);
    return x;
}
__device__ __forceinline__ double wave_max(double x)
{
    x = fmax(x, dpp_partner<DPP_QUAD_XOR1>(x));
    x = fmax(x, dpp_partner<DPP_QUAD_XOR2>(x));
    x = fmax(x, dpp_partner<DPP_ROW_HALF_MIRROR>(x));
    x = fmax(x, dpp_partner<DPP_ROW_MIRROR>(x));
    x = fmax(x, __shfl_xor(x, 16, 64));
    x = fmax(x, __shfl_xor(x, 32, 64));
    return x;
}
__device__ __forceinline__ int wave_sum_i(int x)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o, 64);
    return x;
}

// Typed SoA view.
template <typename T> struct V3 {
    T* x; T* y; T* z;
};
template <typename T> inline V3<T> v3(dsmc_vec3 v)
{
    return V3<T>{static_cast<T*>(v.x), static_cast<T*>(v.y), static_cast<T*>(v.z)};
}

// Device-wide exclusive scan of int32 counts into int32 offsets (n+1 outputs:
// out[n] = total); also stores the total as int64 to *total64 when given.
size_t scan_ws_bytes(int64_t n);
int exclusive_scan_i32(const int32_t* in, int32_t* out, int64_t n, int64_t* total64, void* ws,
                       hipStream_t s);
// Same with a device-side element count (n_dev) bounded by n_max.
int exclusive_scan_i32_dev(const int32_t* in, int32_t* out, const int64_t* n_dev, int64_t n_max,
                           void* ws, hipStream_t s);

// Fill kernels (graph-safe replacements of memset).
int fill_i32(int32_t* p, int32_t value, int64_t n, hipStream_t s);
int fill_bytes_zero(void* p, size_t bytes, hipStream_t s);

// Schedule threshold (pairs per cell above which AUTO uses the BLOCK schedule).
int32_t block_threshold();

}  // namespace dsmc
