// common.hpp -- shared device helpers for the gfx950 kernels of libfastfact.
//
// MFMA lane layouts used throughout (checked on gfx950 hardware):
//   v_mfma_f64_16x16x4f64   A (16x4): lane l holds A[l%16][l/16]
//                           B (4x16): lane l holds B[l/16][l%16]
//                           D (16x16, 4 doubles): D[i][j] sits in lane j + 16*(i%4), register i/4
//   v_mfma_f32_16x16x4f32   A, B as above; D[i][j] sits in lane j + 16*(i/4), register i%4
//   v_mfma_f32_16x16x32_bf16
//                           A (16x32): lane l holds A[l%16][8*(l/16) + e], e = 0..7
//                           B (32x16): lane l holds B[8*(l/16) + e][l%16]
//                           D as for f32.
// Every kernel computes the TRANSPOSED product tile D'[a][b] = S[b][a] (a runs
// over output columns, b over output rows) so that the 16 lanes of a lane group
// hold 16 consecutive rows of one output column: column-major global accesses of
// C are then whole 128-byte lines.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace ff {

typedef double d4_t __attribute__((ext_vector_type(4)));
typedef float f4_t __attribute__((ext_vector_type(4)));
typedef __bf16 bf8_t __attribute__((ext_vector_type(8)));

constexpr int WAVE = 64;

__device__ __forceinline__ d4_t mfma_f64(double a, double b, d4_t c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ f4_t mfma_f32(float a, float b, f4_t c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ f4_t mfma_bf16(bf8_t a, bf8_t b, f4_t c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}

// Accumulator traits: which output column of the 16x16 transposed tile a lane's
// register r holds (the row is always lane % 16).
template <typename T> struct acc_traits;
// col = col_lane(lane) + col_reg(r).
template <> struct acc_traits<double> {
    typedef d4_t vec;
    __device__ static __forceinline__ int col(int lane, int r) { return 4 * r + (lane >> 4); }
    __device__ static __forceinline__ int col_lane(int lane) { return lane >> 4; }
    static constexpr int col_reg(int r) { return 4 * r; }
    __device__ static __forceinline__ vec mfma(double a, double b, vec c) { return mfma_f64(a, b, c); }
};
template <> struct acc_traits<float> {
    typedef f4_t vec;
    __device__ static __forceinline__ int col(int lane, int r) { return 4 * (lane >> 4) + r; }
    __device__ static __forceinline__ int col_lane(int lane) { return 4 * (lane >> 4); }
    static constexpr int col_reg(int r) { return r; }
    __device__ static __forceinline__ vec mfma(float a, float b, vec c) { return mfma_f32(a, b, c); }
};

template <typename V> __device__ __forceinline__ V zero_vec() { V v; v[0] = 0; v[1] = 0; v[2] = 0; v[3] = 0; return v; }

// Round binary32 to bfloat16, nearest with ties to even (the hardware conversion).
__device__ __forceinline__ __bf16 to_bf16(float x) { return (__bf16)x; }

// Raw buffer access.  A buffer resource covers [base, base + BUF_RECORDS) bytes;
// a load whose offset lies at or past BUF_RECORDS returns zero and such a store
// is dropped by the hardware.  Kernels point the resource at the corner of the
// tile they touch and send out-of-matrix elements to BUF_OOB, which gives masked
// loads and stores with no branches.  Hosts keep every in-range byte offset
// below BUF_RECORDS.
constexpr int BUF_RECORDS = 0x7FFFFFF0;
constexpr int BUF_OOB = 0x7FFFFFF0;
typedef __amdgpu_buffer_rsrc_t rsrc_t;

__device__ __forceinline__ rsrc_t make_rsrc(const void* base) {
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(base), (short)0, BUF_RECORDS, 0x00020000);
}
// Resource covering [base, base + bytes): accesses at or past `bytes` read zero.
__device__ __forceinline__ rsrc_t make_rsrc_n(const void* base, int bytes) {
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(base), (short)0, bytes, 0x00020000);
}
// off: per-lane byte offset; soff: wave-uniform byte offset (added to off);
// AUX: cache policy (2 = non-temporal, for data streamed once).
template <typename T, int AUX = 0> struct bufop;
template <int AUX> struct bufop<double, AUX> {
    __device__ static __forceinline__ double load(rsrc_t r, int off, int soff) {
        return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, off, soff, AUX));
    }
    __device__ static __forceinline__ void store(rsrc_t r, int off, double v, int soff) {
        typedef unsigned int u2 __attribute__((ext_vector_type(2)));
        __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u2, v), r, off, soff, AUX);
    }
};
template <int AUX> struct bufop<float, AUX> {
    __device__ static __forceinline__ float load(rsrc_t r, int off, int soff) {
        return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, off, soff, AUX));
    }
    __device__ static __forceinline__ void store(rsrc_t r, int off, float v, int soff) {
        __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned int, v), r, off, soff, AUX);
    }
};
template <typename T> __device__ __forceinline__ T buf_load(rsrc_t r, int off, int soff = 0) {
    return bufop<T, 0>::load(r, off, soff);
}
template <typename T> __device__ __forceinline__ void buf_store(rsrc_t r, int off, T v, int soff = 0) {
    bufop<T, 0>::store(r, off, v, soff);
}
constexpr int AUX_NT = 2;

// Row i of the packed triangle index t = i(i+1)/2 + j (0 <= j <= i): a float
// estimate corrected by one step either way (exact for t < 2^20).
__device__ __forceinline__ int tri_row(int t) {
    int i = (int)((sqrtf(8.0f * (float)t + 1.0f) - 1.0f) * 0.5f);
    if ((i + 1) * (i + 2) / 2 <= t) ++i;
    if (i * (i + 1) / 2 > t) --i;
    return i;
}

// Grid geometry of the update kernels: output tiles grouped into square
// super-tiles (8 x 8 tiles for square tiles); every XCD of the chip (workgroups
// are dealt to the 8 XCDs round-robin) works through whole super-tiles so the
// panel blocks a super-tile reads stay in that XCD's L2.
constexpr int UPD_TILE = 128;
constexpr int UPD_GROUP = 8;
constexpr int N_XCD = 8;

}  // namespace ff
