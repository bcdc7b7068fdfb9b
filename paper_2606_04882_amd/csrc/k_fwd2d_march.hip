// 2D forward step for cross stencils on large windows: the block marches
// along z instead of owning a tile.
//
// A block of kBlock3 threads owns kBlock3 consecutive columns x and a chunk
// of `zchunk` rows; each thread keeps the 2M+1 values of u^n along z of its
// column in registers (a queue shifted once per row) and the block stages
// the current row, with an M-cell halo on each side, in LDS for the x
// neighbours (double-buffered: one barrier per row; the operands of row z+1
// are fetched while row z is computed).  Every value of u^n is read once per
// block plus 2M rows per chunk, instead of the 2M halo rows of every
// 4*rows-row tile of k_fwd2d; d^n, v, d^{n+1} and u^{n+1} are streamed
// non-temporally.  The per-point arithmetic is that of the cross path of
// stencil2d (z pairs first, then x pairs, in the difference form) and of
// fwd2d_tile, so results are bitwise those of k_fwd2d.  Selected with one
// row per thread (fd_set_tile rows = 1) for windows wide and tall enough to
// fill the GPU with chunks.
#include "fd_kernels.h"

namespace fdw {

namespace {

template <int M>
__global__ __launch_bounds__(kBlock3) void k_fwd2d_march(StepArgs p) {
    constexpr int NQ = 2 * M + 1;
    constexpr int W = kBlock3, RW = W + 2 * M;
    __shared__ float rows[2][RW];
    if (p.trace_out) {
        for (int r = blockIdx.x * kBlock3 + threadIdx.x; r < p.nrec; r += gridDim.x * kBlock3) {
            const long long i = p.rec_lin[r];
            p.trace_out[r] = i >= 0 ? p.ucur[i] : 0.f;
        }
    }
    const int t = xcd_tile(blockIdx.x, p.ntiles);
    const int bx = t % p.tiles_x, bz = t / p.tiles_x;
    const int tid = threadIdx.x;
    const int x0 = bx * W, zs = bz * p.zchunk, ze = min(zs + p.zchunk, p.nz);
    const int gx = x0 + tid;
    const bool xok = gx < p.nx;
    const long long nx = p.nx;
    float q[NQ];
#pragma unroll
    for (int i = 0; i < 2 * M; ++i) {
        const int z = zs - M + i;
        q[i] = (xok && (unsigned)z < (unsigned)p.nz) ? p.ucur[z * nx + gx] : 0.f;
    }
    // row halo: threads 0..M-1 load x0-M+tid, threads M..2M-1 load x0+W+tid-M
    const bool hthr = tid < 2 * M;
    const int hx = tid < M ? x0 - M + tid : x0 + W + tid - M;
    const bool hok = hthr && (unsigned)hx < (unsigned)p.nx;
    const int hslot = tid < M ? tid : W + tid;
    float front = 0.f, dd = 0.f, vv = 0.f, hv = 0.f;
    auto fetch = [&](int z) {
        const bool in = z < ze;
        const int zz = z + M;
        front = (xok && in && zz < p.nz) ? p.ucur[zz * nx + gx] : 0.f;
        dd = (xok && in) ? __builtin_nontemporal_load(p.dcur + z * nx + gx) : 0.f;
        vv = (xok && in) ? __builtin_nontemporal_load(p.v + z * p.ldv_y + gx) : 0.f;
        hv = (hok && in) ? p.ucur[z * nx + hx] : 0.f;
    };
    const float qs = p.src >= 0 ? p.q * p.wavelet[p.step] : 0.f;
    const int dxb = (p.sp.nb > 0 && xok) ? band_depth(gx, p.nx, p.sp.nb) : 0;
    fetch(zs);
    int buf = 0;
    for (int z = zs; z < ze; ++z) {
        float* row = rows[buf];
        q[2 * M] = front;
        const float ddc = dd, vvc = vv;
        row[M + tid] = q[M];
        if (hthr) row[hslot] = hv;
        fetch(z + 1);
        __syncthreads();
        if (xok) {
            const float u = q[M];
            float acc = 0.f;
#pragma unroll
            for (int dz = 1; dz <= M; ++dz) acc = fmaf(p.w.w[dz], fmaf(-2.f, u, q[M + dz] + q[M - dz]), acc);
#pragma unroll
            for (int dx = 1; dx <= M; ++dx)
                acc = fmaf(p.w.w[dx], fmaf(-2.f, u, row[M + tid - dx] + row[M + tid + dx]), acc);
            const long long k = z * nx + gx;
            const int dzb = p.sp.nb > 0 ? band_depth(z, p.nz, p.sp.nb) : 0;
            const bool inband = (dxb | dzb) != 0;
            float e = 0.f;
            if (inband) {
                const float ex = dxb * p.sp.inv_nb, ez = dzb * p.sp.inv_nb;
                e = p.sp.escale * fmaf(ex, ex, ez * ez);
            }
            const float d = delta_update(ddc, vvc, acc, inband, e, k == p.src, qs);
            __builtin_nontemporal_store(d, p.dnext + k);
            __builtin_nontemporal_store(u + d, p.unext + k);
        }
#pragma unroll
        for (int i = 0; i < 2 * M; ++i) q[i] = q[i + 1];
        buf ^= 1;
    }
}

template <int M>
void run_march(const StepArgs& a, hipStream_t s) {
    hipLaunchKernelGGL((k_fwd2d_march<M>), dim3(a.ntiles), dim3(kBlock3), 0, s, a);
}

}  // namespace

bool launch_fwd2d_march(const StepArgs& a, int M, hipStream_t s) {
    switch (M) {
        case 1: run_march<1>(a, s); return true;
        case 2: run_march<2>(a, s); return true;
        case 3: run_march<3>(a, s); return true;
        case 4: run_march<4>(a, s); return true;
        case 5: run_march<5>(a, s); return true;
        case 6: run_march<6>(a, s); return true;
        case 7: run_march<7>(a, s); return true;
        case 8: run_march<8>(a, s); return true;
    }
    return false;
}

}  // namespace fdw
