// One 2D forward tile (shared by the single-shot and the batched kernels):
// LDS-staged stencil in difference form, leapfrog in difference form
// (d^{n+1}, u^{n+1} from u^n, d^n: see delta_update), damping band, source.
#pragma once

#include "fd_kernels.h"
#include "stencil2d.h"

namespace fdw {

struct Tile2D {
    const float* __restrict__ ucur;  // u^n
    const float* dcur;               // d^n
    float* dnext;                    // d^{n+1} (may equal dcur: each point is read and written by one thread)
    float* unext;                    // u^{n+1}
    const float* __restrict__ v;
    long long ldv;                 // model row stride of v
    int nx, nz;                    // window
    int x0, z0;                    // tile origin
    long long src;                 // source node (window-linear) or -1
    float qs;                      // q * s^n (source term of this step)
};

template <int SHAPE, int M, int RY>
constexpr int tile2d_floats() {
    return (4 * RY + 2 * M) * tile_pitch2d<SHAPE, M>();
}

// SPLIT: take the rows of threads that are wholly inside the damping-free
// interior and away from the source through a separate store loop, testing
// the band and the source per thread rather than per row.  The arithmetic
// is the same either way.  The split form needs fewer registers (cross M8:
// 67 instead of 115 VGPRs in the batched kernel), which lets the variant
// groups of a batched call share the CUs when they run concurrently (the
// 8-stencil 1001^2 step: 74.7 -> 65.5 ms); a kernel running alone is 3-8 %
// slower with it, so the single-shot kernels keep the per-row form.
template <int SHAPE, int M, int RY, bool SPLIT = false>
__device__ __forceinline__ void fwd2d_tile(const Tile2D& t, const Sponge& sp, const Weights& W,
                                           float* tile) {
    constexpr int LW = tile_pitch2d<SHAPE, M>();
    const int tid = threadIdx.x, tx = tid & 63, ty = tid >> 6;
    // pointwise operands first, then the tile: all global loads in flight together
    const int gx = t.x0 + tx;
    const int zr = t.z0 + ty * RY;                      // the thread's first row
    const int nrow = t.nz - zr;                         // rows left in the window
    const bool colok = gx < t.nx;
    const long long base = (long long)zr * t.nx + gx;   // window-linear index of that row
    float dd[RY], vv[RY];
    {
        long long iu = base, iv = (long long)zr * t.ldv + gx;   // row indices, stepped per row
#pragma unroll
        for (int j = 0; j < RY; ++j) {
            dd[j] = 0.f;
            vv[j] = 0.f;
            if (colok && j < nrow) {
                dd[j] = t.dcur[iu];
                vv[j] = t.v[iv];
            }
            iu += t.nx;
            iv += t.ldv;
        }
    }
    load_tile2d<M, RY, LW>(tile, t.ucur, t.nx, t.nz, t.x0, t.z0);
    __syncthreads();

    float uc[RY], acc[RY];
    stencil2d<SHAPE, M, RY, LW>(tile, tx, ty, W, uc, acc);
    if (!colok) return;

    const int dxb = sp.nb > 0 ? band_depth(gx, t.nx, sp.nb) : 0;
    if constexpr (SPLIT) {
        // a source less than RY rows after the thread's first point (in any
        // column) sends the thread through the per-row loop, which tests
        // each of its points
        const long long srel = t.src - base;
        const bool has_src = t.src >= 0 && srel >= 0 && srel < (long long)RY * t.nx;
        const bool interior = sp.nb == 0 || (dxb == 0 && zr >= sp.nb && zr + RY <= t.nz - sp.nb);
        if (interior && !has_src) {
#pragma unroll
            for (int j = 0; j < RY; ++j) {
                if (j >= nrow) break;
                const float d = fmaf(vv[j], acc[j], dd[j]);
                t.dnext[base + (long long)j * t.nx] = d;
                t.unext[base + (long long)j * t.nx] = uc[j] + d;
            }
            return;
        }
    }
#pragma unroll
    for (int j = 0; j < RY; ++j) {
        if (j >= nrow) break;
        const int gz = zr + j;
        const long long k = (long long)gz * t.nx + gx;
        const bool at_src = k == t.src;
        const int dzb = sp.nb > 0 ? band_depth(gz, t.nz, sp.nb) : 0;
        const bool inband = (dxb | dzb) != 0;
        float e = 0.f;
        if (inband) {
            const float ex = dxb * sp.inv_nb, ez = dzb * sp.inv_nb;
            e = sp.escale * fmaf(ex, ex, ez * ez);
        }
        const float d = delta_update(dd[j], vv[j], acc[j], inband, e, at_src, t.qs);
        t.dnext[k] = d;
        t.unext[k] = uc[j] + d;
    }
}

}  // namespace fdw
