// dev_curves.h -- Hilbert and Z-Morton orders of cells in a 2^k x 2^k square (x = column,
// y = row), shared by the conversion kernels.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

// Hilbert index of local cell (row y, column x) in a 2^k x 2^k block: the classical
// quadrant-by-quadrant descent (quadrant order q = 0..3 is (x<h,y<h), (x<h,y>=h), (x>=h,y>=h),
// (x>=h,y<h); entering quadrants 0 and 3 transposes / anti-transposes the remaining bits).
__device__ __forceinline__ uint32_t hilbert_xy2d(int k, uint32_t x, uint32_t y) {
    uint32_t d = 0;
    for (int l = k - 1; l >= 0; --l) {
        const uint32_t h = 1u << l;
        const uint32_t rx = (x >> l) & 1u, ry = (y >> l) & 1u;
        d += h * h * ((3u * rx) ^ ry);
        if (ry == 0) {
            if (rx == 1) {  // reflect the low bits through the anti-diagonal
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

// Inverse of hilbert_xy2d: local (x = column, y = row) of index d, built up from the finest
// level, undoing each level's transform.
__device__ __forceinline__ void hilbert_d2xy(int k, uint32_t d, uint32_t* px, uint32_t* py) {
    uint32_t x = 0, y = 0, t = d;
    for (int l = 0; l < k; ++l) {
        const uint32_t h = 1u << l;
        const uint32_t rx = 1u & (t >> 1);
        const uint32_t ry = 1u & (t ^ rx);
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

// Z-Morton index of local cell (row y, column x): bits interleaved with the row bit above the
// column bit at every level (quadrants top-left, top-right, bottom-left, bottom-right).
__device__ __forceinline__ uint32_t zmorton_xy2d(int k, uint32_t x, uint32_t y) {
    uint32_t d = 0;
    for (int l = 0; l < k; ++l)
        d |= (((y >> l) & 1u) << (2 * l + 1)) | (((x >> l) & 1u) << (2 * l));
    return d;
}

__device__ __forceinline__ void zmorton_d2xy(int k, uint32_t d, uint32_t* px, uint32_t* py) {
    uint32_t x = 0, y = 0;
    for (int l = 0; l < k; ++l) {
        x |= ((d >> (2 * l)) & 1u) << l;
        y |= ((d >> (2 * l + 1)) & 1u) << l;
    }
    *px = x;
    *py = y;
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
