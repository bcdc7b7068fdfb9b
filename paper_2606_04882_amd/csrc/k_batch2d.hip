// Batched ragged multi-shot kernels (2D).
//
// Many shots, each a window of its own size into one velocity model with its
// own stencil (shape, M), source and receivers, advance one time step in a
// single launch per stencil variant: the host sorts the shots by variant and
// flattens each variant group's tiles into one work list; each block looks up
// its (shot, tile) pair and runs the same tile body as the single-shot
// kernels with that shot's parameters.  Kernels are compiled per variant, so
// each group runs at its own register and LDS budget.  Tiles are 64 x 16 (4
// rows per thread), or 64 x 32 for the forward steps of a dense-stencil
// group.  Fields are named by slot in each shot's
// arena (see BatchShot), so forward, checkpoint, recompute and adjoint phases
// of all shots of a group share one launch per step.
#include "adj2d_body.h"
#include "fwd2d_body.h"

namespace fdw {

constexpr int kBatchRows = 4;

#define FDW_SWITCH(CASE)                                                                        \
    CASE(SH_CROSS, 1) CASE(SH_CROSS, 2) CASE(SH_CROSS, 3) CASE(SH_CROSS, 4) CASE(SH_CROSS, 5)   \
    CASE(SH_CROSS, 6) CASE(SH_CROSS, 7) CASE(SH_CROSS, 8) CASE(SH_RHOMBUS, 1)                   \
    CASE(SH_RHOMBUS, 2) CASE(SH_RHOMBUS, 3) CASE(SH_RHOMBUS, 4) CASE(SH_RHOMBUS, 5)             \
    CASE(SH_RHOMBUS, 6) CASE(SH_RHOMBUS, 7) CASE(SH_RHOMBUS, 8) CASE(SH_SQUARE, 1)              \
    CASE(SH_SQUARE, 2) CASE(SH_SQUARE, 3) CASE(SH_SQUARE, 4) CASE(SH_SQUARE, 5)                 \
    CASE(SH_SQUARE, 6) CASE(SH_SQUARE, 7) CASE(SH_SQUARE, 8) CASE(SH_NSHAPE, 1)                \
    CASE(SH_NSHAPE, 2) CASE(SH_NSHAPE, 3) CASE(SH_NSHAPE, 4) CASE(SH_NSHAPE, 5)                 \
    CASE(SH_NSHAPE, 6) CASE(SH_NSHAPE, 7) CASE(SH_NSHAPE, 8)

template <int SH, int MM, int RY>
__global__ __launch_bounds__(kBlock) void k_batch2d(BatchArgs p) {
    __shared__ float tile[tile2d_floats<SH, MM, RY>()];
    const int job = xcd_tile(blockIdx.x, p.njobs);
    const int2 jb = p.jobs[job];
    const BatchShot& s = p.shots[jb.x];
    const int lt = jb.y;
    const int n = p.step;
    const float* cur = slot_ptr(s, p.f_ucur);
    if (p.gather && n > 0) {
        float* out = s.traces + (long long)(n - 1) * s.nrec;
        for (int r = lt * kBlock + threadIdx.x; r < s.nrec; r += s.ntiles * kBlock) {
            const long long i = s.rec_lin[r];
            out[r] = i >= 0 ? cur[i] : 0.f;
        }
    }
    Tile2D tl;
    tl.ucur = cur;
    tl.dcur = slot_ptr(s, p.f_dcur);
    tl.dnext = s.arena + (long long)p.f_dnext * s.npts;
    tl.unext = s.arena + (long long)p.f_unext * s.npts;
    tl.v = s.v;
    tl.ldv = s.ldv;
    tl.nx = s.nx;
    tl.nz = s.nz;
    const int tz = lt / s.tiles_x;
    tl.x0 = (lt - tz * s.tiles_x) * kTileX;
    tl.z0 = tz * 4 * RY;
    tl.src = s.src;
    tl.qs = s.src >= 0 ? p.q * s.wavelet[n] : 0.f;
    fwd2d_tile<SH, MM, RY, true>(tl, p.sp, s.w, tile);
}

template <int SH, int MM>
__global__ __launch_bounds__(kBlock) void k_batch_adj2d(BatchAdjArgs p) {
    constexpr int N = tile2d_floats_adj<SH, MM, kBatchRows>();
    __shared__ float tp[N];
    __shared__ float tu[N];
    const int job = xcd_tile(blockIdx.x, p.njobs);
    const int2 jb = p.jobs[job];
    const BatchShot& s = p.shots[jb.x];
    const int lt = jb.y;
    AdjTile a;
    a.pcur = slot_ptr(s, p.f_pcur);
    a.pprev = slot_ptr(s, p.f_pprev);
    a.pnext = p.f_pnext >= 0 ? s.arena + (long long)p.f_pnext * s.npts : nullptr;
    a.ufwd = slot_ptr(s, p.f_ufwd);
    a.v = s.v;
    a.ldv = s.ldv;
    a.grad = s.gacc;
    a.ldg = s.nx;
    a.gscale = p.gscale;
    a.gparam = p.gparam;
    a.nx = s.nx;
    a.nz = s.nz;
    const int tz = lt / s.tiles_x;
    a.x0 = (lt - tz * s.tiles_x) * kTileX;
    a.z0 = tz * 4 * kBatchRows;
    a.with_grad = p.with_grad && a.ufwd != nullptr;
    a.with_update = p.with_update;
    adj2d_tile<SH, MM, kBatchRows>(a, p.sp, s.w, tp, tu);
}

// dst <- src per shot; blockIdx.y = shot
__global__ void k_batch_copy(const BatchShot* __restrict__ shots, int dst, int src) {
    const BatchShot& s = shots[blockIdx.y];
    float* d = dst == SLOT_GACC ? s.gacc
             : dst <= SLOT_CKPT0 ? (s.ckpt ? s.ckpt + (long long)(SLOT_CKPT0 - dst) * s.npts : nullptr)
                                 : s.arena + (long long)dst * s.npts;
    if (!d) return;
    const float* a = slot_ptr(s, src);
    for (long long i = blockIdx.x * (long long)kBlock + threadIdx.x; i < s.npts;
         i += (long long)gridDim.x * kBlock)
        d[i] = a ? a[i] : 0.f;
}

__global__ void k_batch_inject(const BatchShot* __restrict__ shots, int f, int k, Sponge sp) {
    const BatchShot& s = shots[blockIdx.y];
    float* psi = s.arena + (long long)f * s.npts;
    const float* rho = s.trace_adj + (long long)(k - 1) * s.nrec;
    for (int r = blockIdx.x * kBlock + threadIdx.x; r < s.nrec; r += gridDim.x * kBlock) {
        const long long i = s.rec_lin[r];
        if (i < 0) continue;
        const int x = (int)(i % s.nx), z = (int)(i / s.nx);
        const float vv = s.v[(long long)z * s.ldv + x];
        float e = 0.f;
        if (sp.nb > 0) {
            const float rx = band_depth(x, s.nx, sp.nb) * sp.inv_nb;
            const float rz = band_depth(z, s.nz, sp.nb) * sp.inv_nb;
            e = sp.escale * fmaf(rx, rx, rz * rz);
        }
        atomicAdd(&psi[i], vv * rho[r] / (1.f + e));
    }
}

__global__ void k_batch_gather(const BatchShot* __restrict__ shots, int f, int n) {
    const BatchShot& s = shots[blockIdx.y];
    const float* u = s.arena + (long long)f * s.npts;
    for (int r = blockIdx.x * kBlock + threadIdx.x; r < s.nrec; r += gridDim.x * kBlock) {
        const long long i = s.rec_lin[r];
        s.traces[(long long)n * s.nrec + r] = i >= 0 ? u[i] : 0.f;
    }
}

int batch_rows() { return kBatchRows; }

bool launch_batch2d(const BatchArgs& a, int shape, int M, int rows, hipStream_t s) {
    if (a.njobs <= 0) return true;
    if (rows == 8) {
        if (shape == SH_CROSS) return false;
        switch (shape * 8 + M - 1) {
#define FDW_CASE(SH, MM)                                                                      \
    case SH * 8 + MM - 1:                                                                     \
        if constexpr (SH != SH_CROSS)                                                         \
            hipLaunchKernelGGL((k_batch2d<SH, MM, 8>), dim3(a.njobs), dim3(kBlock), 0, s, a); \
        return true;
            FDW_SWITCH(FDW_CASE)
#undef FDW_CASE
            default: return false;
        }
    }
    if (rows != kBatchRows) return false;
    switch (shape * 8 + M - 1) {
#define FDW_CASE(SH, MM)                                                                      \
    case SH * 8 + MM - 1:                                                                     \
        hipLaunchKernelGGL((k_batch2d<SH, MM, kBatchRows>), dim3(a.njobs), dim3(kBlock), 0, s, a); \
        return true;
        FDW_SWITCH(FDW_CASE)
#undef FDW_CASE
        default: return false;
    }
}

bool launch_batch_adj2d(const BatchAdjArgs& a, int shape, int M, hipStream_t s) {
    if (a.njobs <= 0) return true;
    switch (shape * 8 + M - 1) {
#define FDW_CASE(SH, MM)                                                                      \
    case SH * 8 + MM - 1:                                                                     \
        hipLaunchKernelGGL((k_batch_adj2d<SH, MM>), dim3(a.njobs), dim3(kBlock), 0, s, a);    \
        return true;
        FDW_SWITCH(FDW_CASE)
#undef FDW_CASE
        default: return false;
    }
}

void launch_batch_copy(const BatchShot* shots, int nshots, long long max_npts, int dst, int src,
                       hipStream_t s) {
    long long bx = (max_npts + kBlock - 1) / kBlock;
    if (bx > 1024) bx = 1024;
    if (bx < 1) bx = 1;
    hipLaunchKernelGGL(k_batch_copy, dim3((unsigned)bx, nshots), dim3(kBlock), 0, s, shots, dst, src);
}

void launch_batch_inject(const BatchShot* shots, int nshots, int max_nrec, int f, int k, Sponge sp,
                         hipStream_t s) {
    if (max_nrec <= 0) return;
    const int bx = (max_nrec + kBlock - 1) / kBlock;
    hipLaunchKernelGGL(k_batch_inject, dim3(bx, nshots), dim3(kBlock), 0, s, shots, f, k, sp);
}

void launch_batch_gather(const BatchShot* shots, int nshots, int max_nrec, int f, int n, hipStream_t s) {
    if (max_nrec <= 0) return;
    const int bx = (max_nrec + kBlock - 1) / kBlock;
    hipLaunchKernelGGL(k_batch_gather, dim3(bx, nshots), dim3(kBlock), 0, s, shots, f, n);
}

}  // namespace fdw
