// 2D forward step: shaped stencil + leapfrog + damping band + source, with
// the receiver gather of the previous step fused in.
//
//   u^{n+1} = b [ 2 u^n - a u^{n-1} + v (W * u^n) + q s^n delta_{x,xs} ]
//
// (Sec. 3.1 eq. wave_eq with the damping term of Sec. 3.1; Sec. 3.2
// eqs. spacexz_derivative2_sym and time_derivative1), evaluated in
// difference form on the state (u^n, d^n) (see delta_update).  One launch
// per step; u^n is read-only during the launch, so the receiver samples of
// u^n (the trace of step n-1) are gathered here as well; d^{n+1} may
// overwrite d^n in place (each point's d^n is read only by its own thread),
// u^{n+1} goes to a second buffer.
//
// Memory traffic per point: read u^n (plus halo, from L2), d^n, v; write
// d^{n+1}, u^{n+1}: 20 B (16 B is the algorithmic minimum of the scheme; the
// extra write keeps the difference d at full precision).
#include "fwd2d_body.h"

namespace fdw {

template <int SHAPE, int M, int RY>
__global__ __launch_bounds__(kBlock) void k_fwd2d(StepArgs p) {
    __shared__ float tile[tile2d_floats<SHAPE, M, RY>()];
    if (p.trace_out) {
        for (int r = blockIdx.x * kBlock + threadIdx.x; r < p.nrec; r += gridDim.x * kBlock) {
            const long long i = p.rec_lin[r];
            p.trace_out[r] = i >= 0 ? p.ucur[i] : 0.f;
        }
    }
    const int t = xcd_tile(blockIdx.x, p.ntiles);
    const int bz = t / p.tiles_x, bx = t - bz * p.tiles_x;
    Tile2D tl;
    tl.ucur = p.ucur;
    tl.dcur = p.dcur;
    tl.dnext = p.dnext;
    tl.unext = p.unext;
    tl.v = p.v;
    tl.ldv = p.ldv_y;
    tl.nx = p.nx;
    tl.nz = p.nz;
    tl.x0 = bx * kTileX;
    tl.z0 = bz * 4 * RY;
    tl.src = p.src;
    tl.qs = p.src >= 0 ? p.q * p.wavelet[p.step] : 0.f;
    fwd2d_tile<SHAPE, M, RY>(tl, p.sp, p.w, tile);
}

template <int SHAPE, int M, int RY>
static void run(const StepArgs& a, hipStream_t s) {
    hipLaunchKernelGGL((k_fwd2d<SHAPE, M, RY>), dim3(a.ntiles), dim3(kBlock), 0, s, a);
}

template <int SHAPE, int M>
static bool dispatch_rows(const StepArgs& a, int rows, hipStream_t s) {
    switch (rows) {
        case 2: run<SHAPE, M, 2>(a, s); return true;
        case 4: run<SHAPE, M, 4>(a, s); return true;
        case 8: run<SHAPE, M, 8>(a, s); return true;
        default: return false;
    }
}

template <int SHAPE>
static bool dispatch_m(const StepArgs& a, int M, int rows, hipStream_t s) {
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

bool have_fwd2d(int shape, int M, int rows) {
    if (rows == 1) return shape == SH_CROSS && M >= 1 && M <= 8;   // k_fwd2d_march
    return shape >= 0 && shape <= 3 && M >= 1 && M <= 8 && (rows == 2 || rows == 4 || rows == 8);
}

bool launch_fwd2d(const StepArgs& a, int shape, int M, int rows, hipStream_t s) {
    if (rows == 1) return shape == SH_CROSS && launch_fwd2d_march(a, M, s);
    switch (shape) {
        case SH_CROSS: return dispatch_m<SH_CROSS>(a, M, rows, s);
        case SH_RHOMBUS: return dispatch_m<SH_RHOMBUS>(a, M, rows, s);
        case SH_SQUARE: return dispatch_m<SH_SQUARE>(a, M, rows, s);
        case SH_NSHAPE: return dispatch_m<SH_NSHAPE>(a, M, rows, s);
        default: return false;
    }
}

}  // namespace fdw
