// One 2D forward tile (shared by the single-shot and the batched kernels):
// LDS-staged stencil in difference form, leapfrog, damping band, source.
#pragma once

#include "fd_kernels.h"
#include "stencil2d.h"

namespace fdw {

struct Tile2D {
    const float* __restrict__ ucur;
    const float* uprev;
    float* unext;
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

template <int SHAPE, int M, int RY>
__device__ __forceinline__ void fwd2d_tile(const Tile2D& t, const Sponge& sp, const Weights& W,
                                           float* tile) {
    constexpr int LW = tile_pitch2d<SHAPE, M>();
    const int tid = threadIdx.x, tx = tid & 63, ty = tid >> 6;
    // pointwise operands first, then the tile: all global loads in flight together
    const int gx = t.x0 + tx;
    const bool colok = gx < t.nx;
    float up[RY], vv[RY];
#pragma unroll
    for (int j = 0; j < RY; ++j) {
        const int gz = t.z0 + ty * RY + j;
        up[j] = 0.f;
        vv[j] = 0.f;
        if (colok && gz < t.nz) {
            up[j] = t.uprev[(long long)gz * t.nx + gx];
            vv[j] = t.v[(long long)gz * t.ldv + gx];
        }
    }
    load_tile2d<M, RY, LW>(tile, t.ucur, t.nx, t.nz, t.x0, t.z0);
    __syncthreads();

    float uc[RY], acc[RY];
    stencil2d<SHAPE, M, RY, LW>(tile, tx, ty, W, uc, acc);
    if (!colok) return;

    const int dxb = sp.nb > 0 ? band_depth(gx, t.nx, sp.nb) : 0;
#pragma unroll
    for (int j = 0; j < RY; ++j) {
        const int gz = t.z0 + ty * RY + j;
        if (gz >= t.nz) break;
        const long long k = (long long)gz * t.nx + gx;
        const int dzb = sp.nb > 0 ? band_depth(gz, t.nz, sp.nb) : 0;
        float r;
        if ((dxb | dzb) == 0) {
            r = fmaf(vv[j], acc[j], 2.f * uc[j] - up[j]);
            if (k == t.src) r += t.qs;
        } else {
            const float ex = dxb * sp.inv_nb, ez = dzb * sp.inv_nb;
            const float e = sp.escale * fmaf(ex, ex, ez * ez);
            r = fmaf(-(1.f - e), up[j], 2.f * uc[j]);
            r = fmaf(vv[j], acc[j], r);
            if (k == t.src) r += t.qs;
            r = r / (1.f + e);
        }
        t.unext[k] = r;
    }
}

}  // namespace fdw
