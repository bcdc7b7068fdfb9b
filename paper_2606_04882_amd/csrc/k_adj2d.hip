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
#include "adj2d_body.h"

namespace fdw {

template <int SHAPE, int M, int RY>
__global__ __launch_bounds__(kBlock) void k_adj2d(AdjArgs p) {
    constexpr int N = tile2d_floats_adj<SHAPE, M, RY>();
    __shared__ float tp[N];
    __shared__ float tu[N];
    const int t = xcd_tile(blockIdx.x, p.ntiles);
    const int bz = t / p.tiles_x, bx = t - bz * p.tiles_x;
    AdjTile a;
    a.pcur = p.pcur;
    a.pprev = p.pprev;
    a.pnext = p.pnext;
    a.ufwd = p.ufwd;
    a.v = p.v;
    a.ldv = p.ldv_y;
    a.grad = p.grad;
    a.ldg = p.ldv_y;
    a.gscale = p.gscale;
    a.gparam = p.gparam;
    a.nx = p.nx;
    a.nz = p.nz;
    a.x0 = bx * kTileX;
    a.z0 = bz * 4 * RY;
    a.with_grad = p.with_grad;
    a.with_update = p.with_update;
    adj2d_tile<SHAPE, M, RY>(a, p.sp, p.w, tp, tu);
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
        case SH_NSHAPE: return dispatch_m<SH_NSHAPE>(a, M, rows, s);
        default: return false;
    }
}

}  // namespace fdw
