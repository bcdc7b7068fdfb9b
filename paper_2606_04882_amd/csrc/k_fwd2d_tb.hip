// 2D forward, two time steps per launch (temporal blocking).
//
// A block owns a 64 x 4*RY output tile.  It stages u^n on the tile plus a
// 2M halo in LDS, computes u^{n+1} on the tile plus an M halo (step n), keeps
// that in LDS, then computes u^{n+2} on the tile (step n+1).  Both new levels
// are written out of place (u^{n-1}, u^n -> u^{n+1}, u^{n+2}: four buffers
// rotate), because neighbouring blocks still read u^n around their tiles.
// Per two updates the HBM traffic is u^n, u^{n-1}, v once and two writes
// (20 B instead of 32 B), and there is half the number of launches.
//
// Every point is evaluated with exactly the arithmetic of the single-step
// kernel (same groups, same order, same update), so both paths give
// bit-identical fields.
#include "fwd2d_body.h"

namespace fdw {

// Cross stencil sum at LDS position (r, c) of a tile of width LW, in the
// order of stencil2d(): z pairs of the centre column, then x-mirror pairs.
template <int M, int LW>
__device__ __forceinline__ float point_cross(const float* t, int r, int c, const Weights& W, float& uc) {
    const float* p = t + r * LW + c;
    const float u = p[0];
    uc = u;
    float acc = 0.f;
#pragma unroll
    for (int dz = 1; dz <= M; ++dz) {
        const float w = W.w[orbit2(SH_CROSS, M, dz, 0)];
        acc = fmaf(w, fmaf(-2.f, u, p[dz * LW] + p[-dz * LW]), acc);
    }
#pragma unroll
    for (int dx = 1; dx <= M; ++dx) {
        const float w = W.w[orbit2(SH_CROSS, M, dx, 0)];
        acc = fmaf(w, fmaf(-2.f, u, p[-dx] + p[dx]), acc);
    }
    return acc;
}

__device__ __forceinline__ float leapfrog(float uc, float up, float vv, float L, int gx, int gz, int nx,
                                          int nz, const Sponge& sp, bool is_src, float qs) {
    const int dxb = sp.nb > 0 ? band_depth(gx, nx, sp.nb) : 0;
    const int dzb = sp.nb > 0 ? band_depth(gz, nz, sp.nb) : 0;
    float r;
    if ((dxb | dzb) == 0) {
        r = fmaf(vv, L, 2.f * uc - up);
        if (is_src) r += qs;
    } else {
        const float ex = dxb * sp.inv_nb, ez = dzb * sp.inv_nb;
        const float e = sp.escale * fmaf(ex, ex, ez * ez);
        r = fmaf(-(1.f - e), up, 2.f * uc);
        r = fmaf(vv, L, r);
        if (is_src) r += qs;
        r = r / (1.f + e);
    }
    return r;
}

template <int SHAPE, int M, int RY>
__global__ __launch_bounds__(kBlock) void k_fwd2d_tb(TbArgs p) {
    static_assert(SHAPE == SH_CROSS, "two-step kernel is compiled for cross stencils");
    constexpr int TY = 4 * RY;
    constexpr int W0 = kTileX + 4 * M, H0 = TY + 4 * M, N0 = W0 * H0;   // u^n
    constexpr int W1 = kTileX + 2 * M, H1 = TY + 2 * M, N1 = W1 * H1;   // u^{n+1}
    __shared__ float U0[N0];
    __shared__ float U1[N1];
    const int tid = threadIdx.x, tx = tid & 63, ty = tid >> 6;
    // traces n-2 (from u^{n-1}) and n-1 (from u^n)
    if (p.trace_a || p.trace_b) {
        for (int r = blockIdx.x * kBlock + tid; r < p.nrec; r += gridDim.x * kBlock) {
            const long long i = p.rec_lin[r];
            if (p.trace_a) p.trace_a[r] = i >= 0 ? p.uprev[i] : 0.f;
            if (p.trace_b) p.trace_b[r] = i >= 0 ? p.ucur[i] : 0.f;
        }
    }
    const int t = xcd_tile(blockIdx.x, p.ntiles);
    const int bz = t / p.tiles_x, bx = t - bz * p.tiles_x;
    const int x0 = bx * kTileX, z0 = bz * TY;
    const float qs0 = p.src >= 0 ? p.q * p.wavelet[p.step] : 0.f;
    const float qs1 = p.src >= 0 ? p.q * p.wavelet[p.step + 1] : 0.f;

    // Cells are taken column-wise: thread (tx, ty) owns the tile's column tx at
    // rows ty, ty + 4, ... (one index step per row), and the halo columns of a
    // region are spread over the block.
    constexpr int NR1 = (H1 + 3) / 4, NH1 = 2 * M * H1, NHL1 = (NH1 + kBlock - 1) / kBlock;   // step-1 region
    constexpr int NR0 = (H0 + 3) / 4, NH0 = 4 * M * H0, NHL0 = (NH0 + kBlock - 1) / kBlock;   // u^n tile
    const int gx = x0 + tx;
    const bool xok = gx < p.nx;

    // all global loads first: u^{n-1}, v on the step-1 region, v on the tile, u^n with 2M halo
    float up1[NR1 + NHL1], vv1[NR1 + NHL1];
    {
        long long iu = (long long)(z0 - M + ty) * p.nx + gx, iv = (long long)(z0 - M + ty) * p.ldv + gx;
#pragma unroll
        for (int k = 0; k < NR1; ++k) {
            const int r = ty + 4 * k, gz = z0 - M + r;
            up1[k] = 0.f;
            vv1[k] = 0.f;
            if ((NR1 * 4 == H1 || r < H1) && xok && (unsigned)gz < (unsigned)p.nz) {
                up1[k] = p.uprev[iu];
                vv1[k] = p.v[iv];
            }
            iu += 4LL * p.nx;
            iv += 4LL * p.ldv;
        }
#pragma unroll
        for (int k = 0; k < NHL1; ++k) {
            const int i = tid + k * kBlock;
            const int r = i / (2 * M), h = i - r * (2 * M);
            const int gz = z0 - M + r, hx = x0 - M + (h < M ? h : kTileX + h);
            up1[NR1 + k] = 0.f;
            vv1[NR1 + k] = 0.f;
            if ((NHL1 * kBlock == NH1 || i < NH1) && (unsigned)gz < (unsigned)p.nz && (unsigned)hx < (unsigned)p.nx) {
                up1[NR1 + k] = p.uprev[(long long)gz * p.nx + hx];
                vv1[NR1 + k] = p.v[(long long)gz * p.ldv + hx];
            }
        }
    }
    float vv2[RY];
#pragma unroll
    for (int j = 0; j < RY; ++j) {
        const int gz = z0 + ty * RY + j;
        vv2[j] = (xok && gz < p.nz) ? p.v[(long long)gz * p.ldv + gx] : 0.f;
    }
    {
        float val[NR0], hv[NHL0];
        long long iu = (long long)(z0 - 2 * M + ty) * p.nx + gx;
#pragma unroll
        for (int k = 0; k < NR0; ++k) {
            const int r = ty + 4 * k, gz = z0 - 2 * M + r;
            val[k] = 0.f;
            if ((NR0 * 4 == H0 || r < H0) && xok && (unsigned)gz < (unsigned)p.nz) val[k] = p.ucur[iu];
            iu += 4LL * p.nx;
        }
#pragma unroll
        for (int k = 0; k < NHL0; ++k) {
            const int i = tid + k * kBlock;
            const int r = i / (4 * M), h = i - r * (4 * M);
            const int gz = z0 - 2 * M + r, hx = x0 - 2 * M + (h < 2 * M ? h : kTileX + h);
            hv[k] = 0.f;
            if ((NHL0 * kBlock == NH0 || i < NH0) && (unsigned)gz < (unsigned)p.nz && (unsigned)hx < (unsigned)p.nx)
                hv[k] = p.ucur[(long long)gz * p.nx + hx];
        }
#pragma unroll
        for (int k = 0; k < NR0; ++k) {
            const int r = ty + 4 * k;
            if (NR0 * 4 == H0 || r < H0) U0[r * W0 + tx + 2 * M] = val[k];
        }
#pragma unroll
        for (int k = 0; k < NHL0; ++k) {
            const int i = tid + k * kBlock;
            const int r = i / (4 * M), h = i - r * (4 * M);
            if (NHL0 * kBlock == NH0 || i < NH0) U0[r * W0 + (h < 2 * M ? h : kTileX + h)] = hv[k];
        }
    }
    __syncthreads();

    // step n: u^{n+1} on the tile plus an M halo (zero outside the window)
    auto step1 = [&](int r, int c, float up, float vv) {
        const int gz = z0 - M + r, gxx = x0 - M + c;
        float out = 0.f;
        if ((unsigned)gz < (unsigned)p.nz && (unsigned)gxx < (unsigned)p.nx) {
            float uc;
            const float L = point_cross<M, W0>(U0, r + M, c + M, p.w, uc);
            const long long kk = (long long)gz * p.nx + gxx;
            out = leapfrog(uc, up, vv, L, gxx, gz, p.nx, p.nz, p.sp, kk == p.src, qs0);
        }
        U1[r * W1 + c] = out;
    };
#pragma unroll
    for (int k = 0; k < NR1; ++k) {
        const int r = ty + 4 * k;
        if (NR1 * 4 == H1 || r < H1) step1(r, tx + M, up1[k], vv1[k]);
    }
#pragma unroll
    for (int k = 0; k < NHL1; ++k) {
        const int i = tid + k * kBlock;
        const int r = i / (2 * M), h = i - r * (2 * M);
        if (NHL1 * kBlock == NH1 || i < NH1) step1(r, h < M ? h : kTileX + h, up1[NR1 + k], vv1[NR1 + k]);
    }
    __syncthreads();

    // step n+1: u^{n+2} on the tile, with the single-step column kernel's stencil
    float uc[RY], acc[RY];
    stencil2d<SHAPE, M, RY, W1>(U1, tx, ty, p.w, uc, acc);
    if (gx >= p.nx) return;
#pragma unroll
    for (int j = 0; j < RY; ++j) {
        const int gz = z0 + ty * RY + j;
        if (gz >= p.nz) break;
        const long long kk = (long long)gz * p.nx + gx;
        const float un = U0[(ty * RY + j + 2 * M) * W0 + tx + 2 * M];
        p.out1[kk] = uc[j];
        p.out2[kk] = leapfrog(uc[j], un, vv2[j], acc[j], gx, gz, p.nx, p.nz, p.sp, kk == p.src, qs1);
    }
}

template <int SHAPE, int M, int RY>
static void run(const TbArgs& a, hipStream_t s) {
    hipLaunchKernelGGL((k_fwd2d_tb<SHAPE, M, RY>), dim3(a.ntiles), dim3(kBlock), 0, s, a);
}

template <int SHAPE, int M>
static bool rows_tb(const TbArgs& a, int rows, hipStream_t s) {
    switch (rows) {
        case 2: run<SHAPE, M, 2>(a, s); return true;
        case 4: run<SHAPE, M, 4>(a, s); return true;
        default: return false;
    }
}

template <int SHAPE>
static bool m_tb(const TbArgs& a, int M, int rows, hipStream_t s) {
    switch (M) {
        case 1: return rows_tb<SHAPE, 1>(a, rows, s);
        case 2: return rows_tb<SHAPE, 2>(a, rows, s);
        case 3: return rows_tb<SHAPE, 3>(a, rows, s);
        case 4: return rows_tb<SHAPE, 4>(a, rows, s);
        case 5: return rows_tb<SHAPE, 5>(a, rows, s);
        case 6: return rows_tb<SHAPE, 6>(a, rows, s);
        case 7: return rows_tb<SHAPE, 7>(a, rows, s);
        case 8: return rows_tb<SHAPE, 8>(a, rows, s);
        default: return false;
    }
}

bool have_fwd2d_tb(int shape, int M, int rows) {
    return shape == SH_CROSS && M >= 1 && M <= 8 && (rows == 2 || rows == 4);
}

bool launch_fwd2d_tb(const TbArgs& a, int shape, int M, int rows, hipStream_t s) {
    if (!have_fwd2d_tb(shape, M, rows)) return false;
    return m_tb<SH_CROSS>(a, M, rows, s);
}

}  // namespace fdw
