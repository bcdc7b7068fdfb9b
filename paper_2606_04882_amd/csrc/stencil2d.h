// 2D stencil evaluation from an LDS tile, shared by the forward and adjoint
// kernels.
//
// Layout: the block computes a 64 (x) by 4*RY (z) tile; thread (tx, ty)
// owns column x0 + tx and rows z0 + ty*RY .. z0 + ty*RY + RY - 1.  The LDS
// tile holds u over the block tile plus an M-cell halo on every side, row
// major with LW = 64 + 2M floats per row; lanes of a wave read consecutive
// floats, so LDS reads are bank-conflict free.
//
// Arithmetic (difference form, Sec. 3.2 eq. spacexz_derivative2_sym with the
// centre weight eliminated through the r = 0 condition): points are taken in
// symmetric groups {(+-dx, +-dz)} sharing one orbit weight w and
//     L += w * (sum_of_group - |group| * u(x))
// so that every term is a small difference of nearby values; the centre
// weight (large, -sum |o| w_o) never multiplies u directly.  Groups are taken
// dx = 0..M outer, dz inner; x-mirror pairs are summed once per column and
// reused by every output row and every dz.
#pragma once

#include "fd_kernels.h"

namespace fdw {

template <int SHAPE, int M, int RY, int LW, int DZ>
__device__ __forceinline__ void s2_col0(const float* col, const float* uc, float* acc,
                                        const Weights& W) {
    if constexpr (DZ <= M) {
        constexpr int o = orbit2(SHAPE, M, DZ, 0);
        const float w = W.w[o];
#pragma unroll
        for (int j = 0; j < RY; ++j)
            acc[j] = fmaf(w, fmaf(-2.f, uc[j], col[j + M + DZ] + col[j + M - DZ]), acc[j]);
        s2_col0<SHAPE, M, RY, LW, DZ + 1>(col, uc, acc, W);
    }
}

template <int SHAPE, int M, int RY, int MZ, int DX, int DZ>
__device__ __forceinline__ void s2_dz(const float* cs, const float* uc, float* acc,
                                      const Weights& W) {
    if constexpr (DZ <= MZ) {
        constexpr int o = orbit2_of(SHAPE, M, DX, DZ);
        const float w = W.w[o];
#pragma unroll
        for (int j = 0; j < RY; ++j)
            acc[j] = fmaf(w, fmaf(-4.f, uc[j], cs[j + MZ + DZ] + cs[j + MZ - DZ]), acc[j]);
        s2_dz<SHAPE, M, RY, MZ, DX, DZ + 1>(cs, uc, acc, W);
    }
}

template <int SHAPE, int M, int RY, int LW, int DX>
__device__ __forceinline__ void s2_dx(const float* tile, int tx, int ty, const float* uc,
                                      float* acc, const Weights& W) {
    if constexpr (DX <= M) {
        constexpr int MZ = maxdz2(SHAPE, M, DX);
        float cs[RY + 2 * MZ];
#pragma unroll
        for (int j = 0; j < RY + 2 * MZ; ++j) {
            const float* row = tile + (ty * RY + M - MZ + j) * LW + tx + M;
            cs[j] = row[-DX] + row[DX];
        }
        constexpr int o0 = orbit2(SHAPE, M, DX, 0);
        const float w0 = W.w[o0];
#pragma unroll
        for (int j = 0; j < RY; ++j) acc[j] = fmaf(w0, fmaf(-2.f, uc[j], cs[j + MZ]), acc[j]);
        s2_dz<SHAPE, M, RY, MZ, DX, 1>(cs, uc, acc, W);
        s2_dx<SHAPE, M, RY, LW, DX + 1>(tile, tx, ty, uc, acc, W);
    }
}

// Dense shapes (rhombus, square).  For each column offset dx the x second
// difference d(z) = u(x-dx, z) + u(x+dx, z) - 2 u(x, z) is formed once per
// row; the group (dx, dz) then contributes
//     w (d(z+dz) + d(z-dz)) + 2 w (u(x, z+dz) + u(x, z-dz) - 2 u(x, z)),
// and the second part, summed over dx, is folded into the centre column's
// weight wc[dz].  Every term stays a small difference of nearby values, at
// two operations per group instead of three.  W.wd holds the weight of group
// (dx, dz) at wd[dx*(M+1) + dz].
//
// dx runs as a real loop, uniform across the wave, so that only one column
// group of LDS values is live at a time (a fully unrolled form lets the
// compiler hoist every group's reads and exhausts the register file).  The
// square's z extent is M for every dx.  For the rhombus (extent M - dx) each
// iteration branches to a body compiled for its dx (s2_dense_col<DX>), so the
// row range is a constant and the reads are straight-line code with
// immediate offsets (with a run-time extent every read sat behind its own
// branch: 10.6 vs 8.3 us per 1001^2 step at M = 8; the same bodies made the
// square 6 % slower, so it keeps the plain loop).  The cross-rhombus /
// cross-square family (SH_NSHAPE) reads its extent from the stencil's
// W.mz[dx] and differences every row of the tile (no branch on the reads;
// rows beyond the extent are never weighted).
template <int SHAPE, int M, int RY, int LW, int DX>
__device__ __forceinline__ void s2_dense_col(const float* tile, int tx, int ty, float* acc, const Weights& W) {
    constexpr int MZ = M - DX;   // rhombus
    const float* wrow = W.wd + DX * (M + 1);
    float d[RY + 2 * MZ];
#pragma unroll
    for (int j = 0; j < RY + 2 * MZ; ++j) {
        const float* row = tile + (ty * RY + M - MZ + j) * LW + tx + M;
        d[j] = fmaf(-2.f, row[0], row[-DX] + row[DX]);
    }
    const float w0 = wrow[0];
#pragma unroll
    for (int j = 0; j < RY; ++j) acc[j] = fmaf(w0, d[j + MZ], acc[j]);
#pragma unroll
    for (int dz = 1; dz <= MZ; ++dz) {
        const float w = wrow[dz];
#pragma unroll
        for (int j = 0; j < RY; ++j) acc[j] = fmaf(w, d[j + MZ + dz] + d[j + MZ - dz], acc[j]);
    }
}

template <int SHAPE, int M, int RY, int LW>
__device__ __forceinline__ void s2_dense_dx(const float* tile, int tx, int ty, float* acc,
                                            const Weights& W) {
    if constexpr (SHAPE == SH_SQUARE) {
#pragma unroll 1
        for (int dx = 1; dx <= M; ++dx) {
            const float* wrow = W.wd + dx * (M + 1);
            float d[RY + 2 * M];
#pragma unroll
            for (int j = 0; j < RY + 2 * M; ++j) {
                const float* row = tile + (ty * RY + j) * LW + tx + M;
                d[j] = fmaf(-2.f, row[0], row[-dx] + row[dx]);
            }
            const float w0 = wrow[0];
#pragma unroll
            for (int j = 0; j < RY; ++j) acc[j] = fmaf(w0, d[j + M], acc[j]);
#pragma unroll
            for (int dz = 1; dz <= M; ++dz) {
                const float w = wrow[dz];
#pragma unroll
                for (int j = 0; j < RY; ++j) acc[j] = fmaf(w, d[j + M + dz] + d[j + M - dz], acc[j]);
            }
        }
    } else if constexpr (SHAPE == SH_NSHAPE) {
#pragma unroll 1
        for (int dx = 1; dx <= M; ++dx) {
            const int mz = W.mz[dx];
            const float* wrow = W.wd + dx * (M + 1);
            float d[RY + 2 * M];
#pragma unroll
            for (int j = 0; j < RY + 2 * M; ++j) {
                const float* row = tile + (ty * RY + j) * LW + tx + M;
                d[j] = fmaf(-2.f, row[0], row[-dx] + row[dx]);
            }
            const float w0 = wrow[0];
#pragma unroll
            for (int j = 0; j < RY; ++j) acc[j] = fmaf(w0, d[j + M], acc[j]);
#pragma unroll
            for (int dz = 1; dz <= M; ++dz) {
                if (dz <= mz) {
                    const float w = wrow[dz];
#pragma unroll
                    for (int j = 0; j < RY; ++j) acc[j] = fmaf(w, d[j + M + dz] + d[j + M - dz], acc[j]);
                }
            }
        }
    } else {
#pragma unroll 1
        for (int dx = 1; dx <= M; ++dx) {
            switch (dx) {
#define FDW_DENSE_COL(D)                                                                   \
    case D:                                                                                \
        if constexpr (D <= M) s2_dense_col<SHAPE, M, RY, LW, (D <= M ? D : 1)>(tile, tx, ty, acc, W); \
        break;
                FDW_DENSE_COL(1)
                FDW_DENSE_COL(2)
                FDW_DENSE_COL(3)
                FDW_DENSE_COL(4)
                FDW_DENSE_COL(5)
                FDW_DENSE_COL(6)
                FDW_DENSE_COL(7)
                FDW_DENSE_COL(8)
#undef FDW_DENSE_COL
                default:
                    break;
            }
        }
    }
}

// acc[j] = (W * u)(x, z_j) for the thread's RY outputs; uc[j] = u(x, z_j).
template <int SHAPE, int M, int RY, int LW>
__device__ __forceinline__ void stencil2d(const float* tile, int tx, int ty, const Weights& W,
                                          float* uc, float* acc) {
    float col[RY + 2 * M];
#pragma unroll
    for (int j = 0; j < RY + 2 * M; ++j) col[j] = tile[(ty * RY + j) * LW + tx + M];
#pragma unroll
    for (int j = 0; j < RY; ++j) {
        uc[j] = col[j + M];
        acc[j] = 0.f;
    }
    if constexpr (SHAPE == SH_CROSS) {
        s2_col0<SHAPE, M, RY, LW, 1>(col, uc, acc, W);
        s2_dx<SHAPE, M, RY, LW, 1>(tile, tx, ty, uc, acc, W);
    } else {
#pragma unroll
        for (int dz = 1; dz <= M; ++dz) {
            const float w = W.wc[dz];
#pragma unroll
            for (int j = 0; j < RY; ++j)
                acc[j] = fmaf(w, fmaf(-2.f, uc[j], col[j + M + dz] + col[j + M - dz]), acc[j]);
        }
        s2_dense_dx<SHAPE, M, RY, LW>(tile, tx, ty, acc, W);
    }
}

// Row pitch (floats) of a 2D LDS tile.  The square and N-shape kernels, whose
// column loop runs over a run-time offset, pad the rows to 128 floats, a
// multiple of 64 dwords: the reads of one column at successive rows then share
// one address register (row offsets fit the st64 form of the paired LDS read)
// instead of taking a new one every third row (square M8: 2 instead of 20
// address additions per column, 10.33 -> 10.09 us per 1001^2 step).  The
// rhombus bodies, compiled per column offset, are faster unpadded (8.35 vs
// 9.17 us at M8), as are the crosses.
template <int SHAPE, int M>
constexpr int tile_pitch2d() {
    return (SHAPE == SH_SQUARE || SHAPE == SH_NSHAPE) ? 128 : kTileX + 2 * M;
}

// Cooperative load of the (4*RY + 2M) x (64 + 2M) tile of field f (window
// nx x nz, dense rows) with zeros beyond the window, rows LP floats apart.
// Thread (tx, ty) loads column x0 + tx at rows ty, ty + 4, ... (one index
// step of 4 rows per load, coalesced along x); the 2M halo columns are
// spread over the block.  All of a thread's global loads are issued before
// any LDS store, so their latencies overlap instead of adding up.
template <int M, int RY, int LP = kTileX + 2 * M>
__device__ __forceinline__ void load_tile2d(float* tile, const float* __restrict__ f, int nx,
                                            int nz, int x0, int z0) {
    constexpr int LH = 4 * RY + 2 * M;
    constexpr int NR = (LH + 3) / 4;                       // rows per thread, main columns
    constexpr int NH = 2 * M * LH;                         // halo cells
    constexpr int NHL = (NH + kBlock - 1) / kBlock;        // halo cells per thread
    const int tid = threadIdx.x, tx = tid & 63, ty = tid >> 6;
    const int gx = x0 + tx;
    const bool xok = gx < nx;
    const long long step = 4LL * nx;
    long long idx = (long long)(z0 - M + ty) * nx + gx;   // index of the thread's k-th row
    float val[NR];
#pragma unroll
    for (int k = 0; k < NR; ++k) {
        const int r = ty + 4 * k, gz = z0 - M + r;
        val[k] = 0.f;
        if ((NR * 4 == LH || r < LH) && xok && (unsigned)gz < (unsigned)nz) val[k] = f[idx];
        idx += step;
    }
    float hv[NHL];
    int hoff[NHL];
#pragma unroll
    for (int k = 0; k < NHL; ++k) {
        const int i = tid + k * kBlock;
        const int r = i / (2 * M), h = i - r * (2 * M);
        const int c = h < M ? h : kTileX + h;              // tile column
        const int gz = z0 - M + r, hx = x0 - M + c;
        hv[k] = 0.f;
        hoff[k] = r * LP + c;
        if ((NHL * kBlock == NH || i < NH) && (unsigned)gz < (unsigned)nz && (unsigned)hx < (unsigned)nx)
            hv[k] = f[(long long)gz * nx + hx];
    }
#pragma unroll
    for (int k = 0; k < NR; ++k) {
        const int r = ty + 4 * k;
        if (NR * 4 == LH || r < LH) tile[r * LP + tx + M] = val[k];
    }
#pragma unroll
    for (int k = 0; k < NHL; ++k) {
        const int i = tid + k * kBlock;
        if (NHL * kBlock == NH || i < NH) tile[hoff[k]] = hv[k];
    }
}

}  // namespace fdw
