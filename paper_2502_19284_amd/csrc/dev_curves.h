// dev_curves.h -- Hilbert and Z-Morton orders of cells in a 2^k x 2^k square (x = column,
// y = row), shared by the conversion kernels.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

// Hilbert order of the cells of a 2^k x 2^k block (x = column, y = row), k <= 16: the classical
// quadrant-by-quadrant descent.  At each level, with h = 2^l and (rx, ry) the level's bits of
// the (transformed) coordinates, the quadrant digit is (3 rx) ^ ry (quadrant order (x<h,y<h),
// (x<h,y>=h), (x>=h,y>=h), (x>=h,y<h)); entering a quadrant with ry = 0 transposes the lower
// bits, and with rx = 1 as well complements them first (a reflection through the
// anti-diagonal).
//
// The transform in force is one of four (swap sw, complement cm; the two commute and are their
// own inverses), so each level is a lookup in a 16-entry table indexed by (state, 2-bit input),
// giving 2 output bits and the next state.  The tables are generated below from the rule above.
namespace hil {
// state st = sw | cm << 1; raw bit pair q = bx << 1 | by (column bit, row bit)
constexpr uint32_t enc_entry(int st, int q) {  // digit | next state << 2
    int bx = q >> 1, by = q & 1;
    if (st & 1) {
        const int t = bx;
        bx = by;
        by = t;
    }
    if (st & 2) {
        bx ^= 1;
        by ^= 1;
    }
    const int digit = (3 * bx) ^ by;
    int nst = st;
    if (by == 0) nst ^= 1 | (bx << 1);
    return (uint32_t)(digit | (nst << 2));
}
constexpr uint32_t dec_entry(int st, int digit) {  // raw bit pair | next state << 2
    const int tx = digit >> 1, ty = (digit ^ (3 * tx)) & 1;  // transformed bits of the digit
    int bx = tx, by = ty;
    if (st & 2) {  // the transform is its own inverse
        bx ^= 1;
        by ^= 1;
    }
    if (st & 1) {
        const int t = bx;
        bx = by;
        by = t;
    }
    int nst = st;
    if (ty == 0) nst ^= 1 | (tx << 1);
    return (uint32_t)(((bx << 1) | by) | (nst << 2));
}
constexpr uint32_t pack(bool dec, int shift) {  // 2-bit field `shift` of the 16 entries
    uint32_t t = 0;
    for (int i = 0; i < 16; ++i)
        t |= ((dec ? dec_entry(i >> 2, i & 3) : enc_entry(i >> 2, i & 3)) >> shift & 3u)
             << (2 * i);
    return t;
}
constexpr uint32_t ENC_DIGIT = pack(false, 0), ENC_NEXT = pack(false, 2);
constexpr uint32_t DEC_BITS = pack(true, 0), DEC_NEXT = pack(true, 2);

// bits 0..15 of v spread to the even bit positions
__device__ __forceinline__ uint32_t spread16(uint32_t v) {
    v &= 0xFFFFu;
    v = (v | (v << 8)) & 0x00FF00FFu;
    v = (v | (v << 4)) & 0x0F0F0F0Fu;
    v = (v | (v << 2)) & 0x33333333u;
    v = (v | (v << 1)) & 0x55555555u;
    return v;
}
// even bit positions of v packed into bits 0..15
__device__ __forceinline__ uint32_t compact16(uint32_t v) {
    v &= 0x55555555u;
    v = (v | (v >> 1)) & 0x33333333u;
    v = (v | (v >> 2)) & 0x0F0F0F0Fu;
    v = (v | (v >> 4)) & 0x00FF00FFu;
    v = (v | (v >> 8)) & 0x0000FFFFu;
    return v;
}
}  // namespace hil

// Hilbert index of local cell (row y, column x), 0 <= x, y < 2^k.
__device__ __forceinline__ uint32_t hilbert_xy2d(int k, uint32_t x, uint32_t y) {
    const uint32_t q = (hil::spread16(x) << 1) | hil::spread16(y);  // level l at bits 2l, 2l+1
    uint32_t d = 0, st = 0;
    for (int l = k - 1; l >= 0; --l) {
        const uint32_t i2 = (st << 3) | (((q >> (2 * l)) & 3u) << 1);
        d = (d << 2) | ((hil::ENC_DIGIT >> i2) & 3u);
        st = (hil::ENC_NEXT >> i2) & 3u;
    }
    return d;
}

// Inverse of hilbert_xy2d: local (x = column, y = row) of index d < 4^k.
__device__ __forceinline__ void hilbert_d2xy(int k, uint32_t d, uint32_t* px, uint32_t* py) {
    uint32_t q = 0, st = 0;
    for (int l = k - 1; l >= 0; --l) {
        const uint32_t i2 = (st << 3) | (((d >> (2 * l)) & 3u) << 1);
        q = (q << 2) | ((hil::DEC_BITS >> i2) & 3u);
        st = (hil::DEC_NEXT >> i2) & 3u;
    }
    *px = hil::compact16(q >> 1);
    *py = hil::compact16(q);
}

// Z-Morton index of local cell (row y, column x), k <= 16: bits interleaved with the row bit above
// the column bit at every level (quadrants top-left, top-right, bottom-left, bottom-right).
__device__ __forceinline__ uint32_t zmorton_xy2d(int k, uint32_t x, uint32_t y) {
    const uint32_t mask = k >= 16 ? 0xFFFFu : (1u << k) - 1u;
    return hil::spread16(x & mask) | (hil::spread16(y & mask) << 1);
}

__device__ __forceinline__ void zmorton_d2xy(int k, uint32_t d, uint32_t* px, uint32_t* py) {
    const uint32_t mask = k >= 16 ? 0xFFFFu : (1u << k) - 1u;
    *px = hil::compact16(d) & mask;
    *py = hil::compact16(d >> 1) & mask;
}

// The same curve over 64-bit indices (levels up to 31), for orders over whole matrices.
__device__ __forceinline__ uint64_t hilbert_xy2d64(int k, uint32_t x, uint32_t y) {
    uint64_t d = 0;
    for (int l = k - 1; l >= 0; --l) {
        const uint32_t h = 1u << l;
        const uint32_t rx = (x >> l) & 1u, ry = (y >> l) & 1u;
        d += ((uint64_t)h * h) * ((3u * rx) ^ ry);
        if (ry == 0) {
            if (rx == 1) {
                x = (h - 1) - (x & (h - 1));
                y = (h - 1) - (y & (h - 1));
            }
            const uint32_t t = x;
            x = y;
            y = t;
        }
    }
    return d;
}

__device__ __forceinline__ void hilbert_d2xy64(int k, uint64_t d, uint32_t* px, uint32_t* py) {
    uint32_t x = 0, y = 0;
    uint64_t t = d;
    for (int l = 0; l < k; ++l) {
        const uint32_t h = 1u << l;
        const uint32_t rx = (uint32_t)(1u & (t >> 1));
        const uint32_t ry = (uint32_t)(1u & (t ^ rx));
        if (ry == 0) {
            if (rx == 1) {
                x = (h - 1) - x;
                y = (h - 1) - y;
            }
            const uint32_t tmp = x;
            x = y;
            y = tmp;
        }
        x += h * rx;
        y += h * ry;
        t >>= 2;
    }
    *px = x;
    *py = y;
}
