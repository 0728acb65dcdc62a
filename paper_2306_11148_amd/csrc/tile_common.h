// Device helpers shared by the matrix-core tile kernels.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace moa {

typedef __bf16 bf16x2_t __attribute__((ext_vector_type(2)));
typedef __bf16 bf16x8_t __attribute__((ext_vector_type(8)));
typedef float f32x4_t __attribute__((ext_vector_type(4)));
typedef float f32x16_t __attribute__((ext_vector_type(16)));
typedef int i32x8_t __attribute__((ext_vector_type(8)));

// Workgroups are handed to the 8 XCDs round-robin (workgroup id mod 8). Give
// each XCD one contiguous range of tile ids so that the tiles sharing rows of
// A and columns of B run under the same L2. Bijective for any tile count.
__device__ __forceinline__ int xcd_remap(int bid, int total) {
    const int q = total / 8, r = total % 8;
    const int xcd = bid % 8, local = bid / 8;
    return xcd * q + (xcd < r ? xcd : r) + local;
}

// Tile id -> (row block, column block), walking column blocks inside bands
// of `group_m` row blocks so that consecutive tiles reuse the same B columns
// and a few A rows (the L2-sized "dimension lift" of the whole matrix).
__device__ __forceinline__ void tile_coords(int id, int tiles_m, int tiles_n, int group_m,
                                            int *tm, int *tn) {
    const int per_group = group_m * tiles_n;
    const int g = id / per_group;
    const int first = g * group_m;
    const int rows = min(tiles_m - first, group_m);
    const int in = id - g * per_group;
    *tm = first + in % rows;
    *tn = in / rows;
}

// x -> (hi, lo): hi = RNE_bf16(x), lo = RNE_bf16(x - hi). x - hi is exact in
// FP32 (hi keeps the leading 8 significant bits of x), so lo is the BF16
// nearest to the exact residual. Two values per packed 32-bit word.
// The FP32 value of a BF16 is its 16 bits followed by 16 zero bits, so hi is
// widened straight from the packed word (one conversion per pair; the low
// half moves up with a byte permute, which the compiler otherwise turns into
// a second conversion).
__device__ __forceinline__ void split_pair(float x0, float x1, uint32_t *hi, uint32_t *lo) {
    const bf16x2_t h = {(__bf16)x0, (__bf16)x1};
    const uint32_t hw = __builtin_bit_cast(uint32_t, h);
    const float r0 = x0 - __builtin_bit_cast(float, __builtin_amdgcn_perm(0u, hw, 0x01000C0Cu));
    const float r1 = x1 - __builtin_bit_cast(float, hw & 0xFFFF0000u);
    const bf16x2_t l = {(__bf16)r0, (__bf16)r1};
    *hi = hw;
    *lo = __builtin_bit_cast(uint32_t, l);
}

// Output element (row, col) of a 32x32 matrix-core block held in register r
// of lane l: row = 8*(r/4) + 4*(l/32) + r%4, col = l%32.
__device__ __forceinline__ int mfma32_row(int r, int lane) {
    return 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3);
}

}  // namespace moa
