// Batched ragged multi-shot forward step (2D).
//
// Many shots, each a window of its own size into one velocity model with its
// own stencil (shape, M), source and receivers, advance one time step in a
// single launch: the host flattens every shot's tiles into one work list and
// each block looks up its (shot, tile) pair, then runs the same tile body as
// the single-shot kernel with that shot's parameters.  The stencil branch is
// uniform per block.  Tiles are 64 x 16 (4 rows per thread) for every shot.
#include "fwd2d_body.h"

namespace fdw {

constexpr int kBatchRows = 4;

__global__ __launch_bounds__(kBlock) void k_batch2d(BatchArgs p) {
    __shared__ float tile[tile2d_floats<SH_SQUARE, 8, kBatchRows>()];
    const int job = xcd_tile(blockIdx.x, p.njobs);
    const int2 jb = p.jobs[job];
    const BatchShot& s = p.shots[jb.x];
    const int lt = jb.y;
    const int n = p.step;
    const float* cur = s.buf[(n + 1) & 1];
    float* nxt = s.buf[n & 1];
    if (n > 0) {
        float* out = s.traces + (long long)(n - 1) * s.nrec;
        for (int r = lt * kBlock + threadIdx.x; r < s.nrec; r += s.ntiles * kBlock) {
            const long long i = s.rec_lin[r];
            out[r] = i >= 0 ? cur[i] : 0.f;
        }
    }
    Tile2D tl;
    tl.ucur = cur;
    tl.uprev = nxt;
    tl.unext = nxt;
    tl.v = s.v;
    tl.ldv = s.ldv;
    tl.nx = s.nx;
    tl.nz = s.nz;
    const int tz = lt / s.tiles_x;
    tl.x0 = (lt - tz * s.tiles_x) * kTileX;
    tl.z0 = tz * 4 * kBatchRows;
    tl.src = s.src;
    tl.qs = s.src >= 0 ? p.q * s.wavelet[n] : 0.f;
    switch (s.variant) {
#define FDW_CASE(SH, MM) \
    case SH * 8 + MM - 1: fwd2d_tile<SH, MM, kBatchRows>(tl, p.sp, s.w, tile); break;
        FDW_CASE(SH_CROSS, 1) FDW_CASE(SH_CROSS, 2) FDW_CASE(SH_CROSS, 3) FDW_CASE(SH_CROSS, 4)
        FDW_CASE(SH_CROSS, 5) FDW_CASE(SH_CROSS, 6) FDW_CASE(SH_CROSS, 7) FDW_CASE(SH_CROSS, 8)
        FDW_CASE(SH_RHOMBUS, 1) FDW_CASE(SH_RHOMBUS, 2) FDW_CASE(SH_RHOMBUS, 3) FDW_CASE(SH_RHOMBUS, 4)
        FDW_CASE(SH_RHOMBUS, 5) FDW_CASE(SH_RHOMBUS, 6) FDW_CASE(SH_RHOMBUS, 7) FDW_CASE(SH_RHOMBUS, 8)
        FDW_CASE(SH_SQUARE, 1) FDW_CASE(SH_SQUARE, 2) FDW_CASE(SH_SQUARE, 3) FDW_CASE(SH_SQUARE, 4)
        FDW_CASE(SH_SQUARE, 5) FDW_CASE(SH_SQUARE, 6) FDW_CASE(SH_SQUARE, 7) FDW_CASE(SH_SQUARE, 8)
#undef FDW_CASE
        default: break;
    }
}

int batch_rows() { return kBatchRows; }

void launch_batch2d(const BatchArgs& a, hipStream_t s) {
    hipLaunchKernelGGL(k_batch2d, dim3(a.njobs), dim3(kBlock), 0, s, a);
}

}  // namespace fdw
