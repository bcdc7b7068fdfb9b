// One 2D adjoint tile (shared by the single-shot and the batched kernels):
//     psi^k = b [ 2 psi^{k+1} - a psi^{k+2} + v (W * psi^{k+1}) ]
//     grad += f psi^{k+1} (W * u^k),   f = grad_factor(gparam, gscale, v)
//     (f = 2/c for the gradient in the velocity)
#pragma once

#include "fd_kernels.h"
#include "stencil2d.h"

namespace fdw {

template <int SHAPE, int M, int RY>
constexpr int tile2d_floats_adj() {
    return (4 * RY + 2 * M) * tile_pitch2d<SHAPE, M>();
}

struct AdjTile {
    const float* __restrict__ pcur;   // psi^{k+1}
    const float* pprev;               // psi^{k+2}
    float* pnext;                     // psi^k
    const float* __restrict__ ufwd;   // u^k
    const float* __restrict__ v;
    long long ldv;                    // row stride of v
    float* grad;
    long long ldg;                    // row stride of grad
    float gscale;
    int gparam;
    int nx, nz, x0, z0;
    int with_grad, with_update;
};

template <int SHAPE, int M, int RY>
__device__ __forceinline__ void adj2d_tile(const AdjTile& t, const Sponge& sp, const Weights& W,
                                           float* tp, float* tu) {
    constexpr int LW = tile_pitch2d<SHAPE, M>();
    const int tid = threadIdx.x, tx = tid & 63, ty = tid >> 6;
    const int gx = t.x0 + tx;
    const bool colok = gx < t.nx;
    float pp[RY], vv[RY], gg[RY];
#pragma unroll
    for (int j = 0; j < RY; ++j) {
        const int gz = t.z0 + ty * RY + j;
        pp[j] = 0.f;
        vv[j] = 0.f;
        gg[j] = 0.f;
        if (colok && gz < t.nz) {
            if (t.with_update) pp[j] = t.pprev[(long long)gz * t.nx + gx];
            vv[j] = t.v[(long long)gz * t.ldv + gx];
            if (t.with_grad) gg[j] = t.grad[(long long)gz * t.ldg + gx];
        }
    }
    load_tile2d<M, RY, LW>(tp, t.pcur, t.nx, t.nz, t.x0, t.z0);
    if (t.with_grad) load_tile2d<M, RY, LW>(tu, t.ufwd, t.nx, t.nz, t.x0, t.z0);
    __syncthreads();

    float pc[RY], lp[RY];
    stencil2d<SHAPE, M, RY, LW>(tp, tx, ty, W, pc, lp);
    float uc[RY], lu[RY];
    if (t.with_grad) {
        stencil2d<SHAPE, M, RY, LW>(tu, tx, ty, W, uc, lu);
    } else {
#pragma unroll
        for (int j = 0; j < RY; ++j) lu[j] = 0.f;
    }
    if (!colok) return;

    const int dxb = sp.nb > 0 ? band_depth(gx, t.nx, sp.nb) : 0;
#pragma unroll
    for (int j = 0; j < RY; ++j) {
        const int gz = t.z0 + ty * RY + j;
        if (gz >= t.nz) break;
        if (t.with_grad)
            t.grad[(long long)gz * t.ldg + gx] = fmaf(grad_factor(t.gparam, t.gscale, vv[j]) * pc[j], lu[j], gg[j]);
        if (!t.with_update) continue;
        const long long k = (long long)gz * t.nx + gx;
        const int dzb = sp.nb > 0 ? band_depth(gz, t.nz, sp.nb) : 0;
        float r;
        if ((dxb | dzb) == 0) {
            r = fmaf(vv[j], lp[j], 2.f * pc[j] - pp[j]);
        } else {
            const float ex = dxb * sp.inv_nb, ez = dzb * sp.inv_nb;
            const float e = sp.escale * fmaf(ex, ex, ez * ez);
            r = fmaf(-(1.f - e), pp[j], 2.f * pc[j]);
            r = fmaf(vv[j], lp[j], r);
            r = r / (1.f + e);
        }
        t.pnext[k] = r;
    }
}

}  // namespace fdw
