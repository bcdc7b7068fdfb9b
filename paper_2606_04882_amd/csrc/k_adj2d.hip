// 2D adjoint step fused with the gradient accumulation.
//
// Adjoint of the forward recursion (the stencil W is symmetric, so the
// adjoint runs the same operator backwards in time):
//     psi^k = b [ 2 psi^{k+1} - a psi^{k+2} + v (W * psi^{k+1}) ]      (+ receiver
//             residuals, injected by a separate small kernel)
//     dJ/dc += (2 / c) psi^{k+1} (W * u^k)
// One launch computes psi^k and the gradient term that pairs psi^{k+1} (read
// only in this launch, residuals already injected) with the forward field u^k.
// 2/c is formed from v as (2 dt / h) / sqrt(v).
//
// Memory traffic per point: psi^{k+1}, u^k (plus halos), psi^{k+2}, v, the
// gradient (read + write), psi^k (write): 28 B.
#include "fd_kernels.h"
#include "stencil2d.h"

namespace fdw {

template <int SHAPE, int M, int RY>
__global__ __launch_bounds__(kBlock) void k_adj2d(AdjArgs p) {
    constexpr int TY = 4 * RY, LW = kTileX + 2 * M, LH = TY + 2 * M;
    __shared__ float tp[LH * LW];
    __shared__ float tu[LH * LW];
    const int tid = threadIdx.x, tx = tid & 63, ty = tid >> 6;
    const int t = xcd_tile(blockIdx.x, p.ntiles);
    const int bz = t / p.tiles_x, bx = t - bz * p.tiles_x;
    const int x0 = bx * kTileX, z0 = bz * TY;
    const int gx = x0 + tx;
    const bool colok = gx < p.nx;
    float pp[RY], vv[RY], gg[RY];
#pragma unroll
    for (int j = 0; j < RY; ++j) {
        const int gz = z0 + ty * RY + j;
        pp[j] = 0.f;
        vv[j] = 0.f;
        gg[j] = 0.f;
        if (colok && gz < p.nz) {
            if (p.with_update) pp[j] = p.pprev[(long long)gz * p.nx + gx];
            vv[j] = p.v[(long long)gz * p.ldv_y + gx];
            if (p.with_grad) gg[j] = p.grad[(long long)gz * p.ldv_y + gx];
        }
    }
    load_tile2d<M, RY>(tp, p.pcur, p.nx, p.nz, x0, z0);
    if (p.with_grad) load_tile2d<M, RY>(tu, p.ufwd, p.nx, p.nz, x0, z0);
    __syncthreads();

    float pc[RY], lp[RY];
    stencil2d<SHAPE, M, RY, LW>(tp, tx, ty, p.w, pc, lp);
    float uc[RY], lu[RY];
    if (p.with_grad) {
        stencil2d<SHAPE, M, RY, LW>(tu, tx, ty, p.w, uc, lu);
    } else {
#pragma unroll
        for (int j = 0; j < RY; ++j) lu[j] = 0.f;
    }
    if (!colok) return;

    const int dxb = p.sp.nb > 0 ? band_depth(gx, p.nx, p.sp.nb) : 0;
#pragma unroll
    for (int j = 0; j < RY; ++j) {
        const int gz = z0 + ty * RY + j;
        if (gz >= p.nz) break;
        if (p.with_grad)
            p.grad[(long long)gz * p.ldv_y + gx] = fmaf(p.gscale * rsqrtf(vv[j]) * pc[j], lu[j], gg[j]);
        if (!p.with_update) continue;
        const long long k = (long long)gz * p.nx + gx;
        const int dzb = p.sp.nb > 0 ? band_depth(gz, p.nz, p.sp.nb) : 0;
        float r;
        if ((dxb | dzb) == 0) {
            r = fmaf(vv[j], lp[j], 2.f * pc[j] - pp[j]);
        } else {
            const float ex = dxb * p.sp.inv_nb, ez = dzb * p.sp.inv_nb;
            const float e = p.sp.escale * fmaf(ex, ex, ez * ez);
            r = fmaf(-(1.f - e), pp[j], 2.f * pc[j]);
            r = fmaf(vv[j], lp[j], r);
            r = r / (1.f + e);
        }
        p.pnext[k] = r;
    }
}

template <int SHAPE, int M, int RY>
static void run(const AdjArgs& a, hipStream_t s) {
    hipLaunchKernelGGL((k_adj2d<SHAPE, M, RY>), dim3(a.ntiles), dim3(kBlock), 0, s, a);
}

template <int SHAPE, int M>
static bool dispatch_rows(const AdjArgs& a, int rows, hipStream_t s) {
    switch (rows) {
        case 2: run<SHAPE, M, 2>(a, s); return true;
        case 4: run<SHAPE, M, 4>(a, s); return true;
        case 8: run<SHAPE, M, 8>(a, s); return true;
        default: return false;
    }
}

template <int SHAPE>
static bool dispatch_m(const AdjArgs& a, int M, int rows, hipStream_t s) {
    switch (M) {
        case 1: return dispatch_rows<SHAPE, 1>(a, rows, s);
        case 2: return dispatch_rows<SHAPE, 2>(a, rows, s);
        case 3: return dispatch_rows<SHAPE, 3>(a, rows, s);
        case 4: return dispatch_rows<SHAPE, 4>(a, rows, s);
        case 5: return dispatch_rows<SHAPE, 5>(a, rows, s);
        case 6: return dispatch_rows<SHAPE, 6>(a, rows, s);
        case 7: return dispatch_rows<SHAPE, 7>(a, rows, s);
        case 8: return dispatch_rows<SHAPE, 8>(a, rows, s);
        default: return false;
    }
}

bool launch_adj2d(const AdjArgs& a, int shape, int M, int rows, hipStream_t s) {
    switch (shape) {
        case SH_CROSS: return dispatch_m<SH_CROSS>(a, M, rows, s);
        case SH_RHOMBUS: return dispatch_m<SH_RHOMBUS>(a, M, rows, s);
        case SH_SQUARE: return dispatch_m<SH_SQUARE>(a, M, rows, s);
        default: return false;
    }
}

}  // namespace fdw
