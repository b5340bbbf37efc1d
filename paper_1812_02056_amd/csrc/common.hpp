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
template <> struct acc_traits<double> {
    typedef d4_t vec;
    __device__ static __forceinline__ int col(int lane, int r) { return 4 * r + (lane >> 4); }
    __device__ static __forceinline__ vec mfma(double a, double b, vec c) { return mfma_f64(a, b, c); }
};
template <> struct acc_traits<float> {
    typedef f4_t vec;
    __device__ static __forceinline__ int col(int lane, int r) { return 4 * (lane >> 4) + r; }
    __device__ static __forceinline__ vec mfma(float a, float b, vec c) { return mfma_f32(a, b, c); }
};

template <typename V> __device__ __forceinline__ V zero_vec() { V v; v[0] = 0; v[1] = 0; v[2] = 0; v[3] = 0; return v; }

// Round binary32 to bfloat16, nearest with ties to even (the hardware conversion).
__device__ __forceinline__ __bf16 to_bf16(float x) { return (__bf16)x; }

// Grid geometry of the update kernels: output tiles of 128 x 128 grouped into
// 8 x 8 super-tiles; every XCD of the chip (workgroups are dealt to the 8 XCDs
// round-robin) works through whole super-tiles so the 16 panel blocks a
// super-tile reads stay in that XCD's L2.
constexpr int UPD_TILE = 128;
constexpr int UPD_GROUP = 8;
constexpr int N_XCD = 8;
constexpr int UPD_WG_PER_SUPER = UPD_GROUP * UPD_GROUP;

}  // namespace ff
