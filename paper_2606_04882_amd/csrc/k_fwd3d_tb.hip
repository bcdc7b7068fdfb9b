// Two time steps per launch for 3D cross stencils (M <= 4): temporal
// blocking of the update of Sec. 3.1-3.2 (the 3D extension noted at the end
// of Sec. 3.1), so that u^n, u^{n-1} and v cross HBM once for two steps.
//
// A block of kWaves3 waves owns a 64 (x) by kWaves3 (y) core column and
// marches along z through `zchunk` planes.  Per plane p it runs two stages:
//
//  A. u^{n+1} at plane p on the core plus an M-cell xy ring (the "extended"
//     tile E): x/y neighbours of u^n from an LDS copy of plane p with a
//     2M-cell ring (double-buffered, prefetched one plane ahead), z
//     neighbours from a register queue of 2M+1 values per E point.  Each
//     thread owns its core point (E point 0) and at most NPT-1 ring points.
//     The result goes to an LDS ring of M+1 extended planes (values off the
//     grid are 0, as the single-step kernels read them) and, for the core
//     points of the block's own planes, to u^{n+1} in HBM.
//  B. u^{n+2} at plane q = p - M on the core: x/y neighbours of u^{n+1} from
//     the LDS ring, z neighbours from a per-thread register queue of the
//     thread's own core column of u^{n+1} (stage A computed it), u^n(q) from
//     the oldest entry of the core u^n queue.
//
// Every value goes through the same operations in the same order as in
// k_fwd3d_cross (compiled with -ffp-contract=off), so two steps per launch
// are bitwise equal to two single-step launches.  The ring points of E are
// computed by every block that borders them (about 1.25x the stage-A work
// of the core for M = 4), and 2M planes per chunk are recomputed by the
// neighbouring chunk: VALU slack of an HBM-bound step pays for halving the
// HBM passes (20 B per point per launch instead of 2 x 16 B).
#include "fd_kernels.h"

namespace fdw {

namespace {

template <int M>
struct GeoTb3 {
    static constexpr int CX = kTileX, CY = kWaves3;               // core: 64 x 8
    static constexpr int EW = CX + 2 * M, EH = CY + 2 * M;        // extended tile (u^{n+1})
    static constexpr int NE = EW * EH;
    static constexpr int NR = NE - CX * CY;                        // ring points of E
    static constexpr int NPT = 1 + (NR + kBlock3 - 1) / kBlock3;   // E points per thread
    static constexpr int IW = CX + 4 * M, IH = CY + 4 * M;        // u^n plane staging
    static constexpr int NI = IW * IH;
    static constexpr int NIL = (NI + kBlock3 - 1) / kBlock3;
};

__device__ __forceinline__ float damp_tb(const Sponge& sp, int gx, int gy, int gz, int nx, int ny, int nz,
                                         bool& inband) {
    if (sp.nb <= 0) {
        inband = false;
        return 0.f;
    }
    const int dx = band_depth(gx, nx, sp.nb), dy = band_depth(gy, ny, sp.nb), dz = band_depth(gz, nz, sp.nb);
    inband = (dx | dy | dz) != 0;
    if (!inband) return 0.f;
    const float rx = dx * sp.inv_nb, ry = dy * sp.inv_nb, rz = dz * sp.inv_nb;
    return sp.escale * fmaf(rx, rx, fmaf(ry, ry, rz * rz));
}

// (W * u) from an xy plane of row width LW and a z queue centred at q[M]; the
// operations and their order are those of the single-step cross kernel.
template <int M, int LW>
__device__ __forceinline__ float cross_sum_w(const float* tile, const float* q, int row, int col,
                                             const Weights& W) {
    const float u = q[M];
    float acc = 0.f;
#pragma unroll
    for (int m = 1; m <= M; ++m) {
        const float s = (tile[row * LW + col - m] + tile[row * LW + col + m]) +
                        (tile[(row - m) * LW + col] + tile[(row + m) * LW + col]) + (q[M - m] + q[M + m]);
        acc = fmaf(W.w[m], fmaf(-6.f, u, s), acc);
    }
    return acc;
}

// the leapfrog update with damping and source, as in the single-step kernel
__device__ __forceinline__ float leap(float uc, float upc, float vvc, float L, bool inband, float e, bool at_src,
                                      float qs) {
    float r;
    if (!inband) {
        r = fmaf(vvc, L, 2.f * uc - upc);
        if (at_src) r += qs;
    } else {
        r = fmaf(-(1.f - e), upc, 2.f * uc);
        r = fmaf(vvc, L, r);
        if (at_src) r += qs;
        r = r / (1.f + e);
    }
    return r;
}

// E coordinates of the thread's k-th E point (k = 0: its core point; then
// ring points in the order top rows, bottom rows, left and right sides)
template <int M>
__device__ __forceinline__ bool e_point(int k, int tid, int& ex, int& ey) {
    using G = GeoTb3<M>;
    if (k == 0) {
        ex = (tid & 63) + M;
        ey = (tid >> 6) + M;
        return true;
    }
    const int r = tid + (k - 1) * kBlock3;
    if (r >= G::NR) return false;
    constexpr int TOP = M * G::EW, SIDE = G::CY * M;
    if (r < TOP) {
        ey = r / G::EW;
        ex = r - ey * G::EW;
    } else if (r < 2 * TOP) {
        const int q = r - TOP;
        ey = M + G::CY + q / G::EW;
        ex = q % G::EW;
    } else {
        const int q = r - 2 * TOP;
        const int side = q / SIDE, w = q - side * SIDE;
        ey = M + w / M;
        ex = (side ? M + G::CX : 0) + w % M;
    }
    return true;
}

template <int M>
__global__ __launch_bounds__(kBlock3) __attribute__((amdgpu_waves_per_eu(4))) void k_fwd3d_cross_tb(Tb3Args p) {
    using G = GeoTb3<M>;
    constexpr int NQ = 2 * M + 1;
    constexpr int NPT = G::NPT;
    __shared__ float ibuf[2][G::NI];
    __shared__ float ring[M + 1][G::NE];
    if (p.nrec > 0 && (p.trace_a || p.trace_b)) {
        for (int r = blockIdx.x * kBlock3 + threadIdx.x; r < p.nrec; r += gridDim.x * kBlock3) {
            const long long i = p.rec_lin[r];
            if (p.trace_a) p.trace_a[r] = i >= 0 ? p.uprev[i] : 0.f;
            if (p.trace_b) p.trace_b[r] = i >= 0 ? p.ucur[i] : 0.f;
        }
    }
    const int tid = threadIdx.x;
    const int t = xcd_tile(blockIdx.x, p.ntiles);
    const int bx = t % p.tiles_x, t2 = t / p.tiles_x;
    const int by = t2 % p.tiles_y, bz = t2 / p.tiles_y;
    const int x0 = bx * G::CX, y0 = by * G::CY;
    const int zs = bz * p.zchunk, ze = min(zs + p.zchunk, p.nz);
    const long long plane = (long long)p.nx * p.ny;

    // per E point: grid coordinates and offset within a plane (the host
    // takes this kernel only for planes of fewer than 2^31 points); the E
    // coordinates are gx - x0 + M, gy - y0 + M
    int gx[NPT], gy[NPT], col[NPT];
    bool ev[NPT], gin[NPT];
    float un[NPT][NQ];
#pragma unroll
    for (int k = 0; k < NPT; ++k) {
        int ex = 0, ey = 0;
        ev[k] = e_point<M>(k, tid, ex, ey);
        gx[k] = x0 - M + ex;
        gy[k] = y0 - M + ey;
        gin[k] = ev[k] && (unsigned)gx[k] < (unsigned)p.nx && (unsigned)gy[k] < (unsigned)p.ny;
        col[k] = gin[k] ? gy[k] * p.nx + gx[k] : 0;
        // planes zs - 2M .. zs - 1 (the first iteration, plane zs - M, adds zs)
#pragma unroll
        for (int i = 0; i < 2 * M; ++i) {
            const int z = zs - 2 * M + i;
            un[k][i] = (gin[k] && (unsigned)z < (unsigned)p.nz) ? p.ucur[z * plane + col[k]] : 0.f;
        }
    }
    float u1[NQ];   // u^{n+1} along z at the core column (stage B)
#pragma unroll
    for (int i = 0; i < NQ; ++i) u1[i] = 0.f;

    float ival[G::NIL], fr[NPT], up[NPT], vv[NPT], vq = 0.f;
    auto fetch = [&](int pz) {
        const bool zin = (unsigned)pz < (unsigned)p.nz;
#pragma unroll
        for (int kk = 0; kk < G::NIL; ++kk) {
            const int i = tid + kk * kBlock3;
            const int r = i / G::IW, c = i - r * G::IW;
            const int yy = y0 - 2 * M + r, xx = x0 - 2 * M + c;
            ival[kk] = (i < G::NI && zin && (unsigned)xx < (unsigned)p.nx && (unsigned)yy < (unsigned)p.ny)
                           ? p.ucur[pz * plane + (long long)yy * p.nx + xx]
                           : 0.f;
        }
#pragma unroll
        for (int k = 0; k < NPT; ++k) {
            const int zz = pz + M;
            fr[k] = (gin[k] && (unsigned)zz < (unsigned)p.nz) ? p.ucur[zz * plane + col[k]] : 0.f;
            if (k == 0) {
                up[k] = (gin[k] && zin) ? __builtin_nontemporal_load(p.uprev + pz * plane + col[k]) : 0.f;
            } else {
                up[k] = (gin[k] && zin) ? p.uprev[pz * plane + col[k]] : 0.f;
            }
            vv[k] = (gin[k] && zin) ? p.v[(long long)pz * p.ldv_z + (long long)gy[k] * p.ldv_y + gx[k]] : 0.f;
        }
        const int qz = pz - M;
        vq = (gin[0] && qz >= zs && qz < ze) ? p.v[(long long)qz * p.ldv_z + (long long)gy[0] * p.ldv_y + gx[0]]
                                             : 0.f;
    };

    const float qs1 = p.q * p.wavelet[p.step];
    const float qs2 = p.q * p.wavelet[p.step + 1];
    fetch(zs - M);
    int buf = 0;
    for (int pz = zs - M; pz < ze + M; ++pz) {
        float* ib = ibuf[buf];
#pragma unroll
        for (int kk = 0; kk < G::NIL; ++kk) {
            const int i = tid + kk * kBlock3;
            if (i < G::NI) ib[i] = ival[kk];
        }
        float upc[NPT], vvc[NPT];
#pragma unroll
        for (int k = 0; k < NPT; ++k) {
            un[k][2 * M] = fr[k];
            upc[k] = up[k];
            vvc[k] = vv[k];
        }
        const float vqc = vq;
        if (pz + 1 < ze + M) fetch(pz + 1);
        __syncthreads();
        // stage A: u^{n+1} at plane pz on the E points
        float* rs = ring[(pz - zs + 2 * M) % (M + 1)];
        const bool zin = (unsigned)pz < (unsigned)p.nz;
#pragma unroll
        for (int k = 0; k < NPT; ++k) {
            if (!ev[k]) continue;
            float r = 0.f;
            if (gin[k] && zin) {
                const float L = cross_sum_w<M, G::IW>(ib, un[k], gy[k] - y0 + 2 * M, gx[k] - x0 + 2 * M, p.w);
                bool inband;
                const float e = damp_tb(p.sp, gx[k], gy[k], pz, p.nx, p.ny, p.nz, inband);
                r = leap(un[k][M], upc[k], vvc[k], L, inband, e, pz * plane + col[k] == p.src, qs1);
            }
            rs[(gy[k] - y0 + M) * G::EW + (gx[k] - x0 + M)] = r;
            if (k == 0) {
                u1[2 * M] = r;
                if (gin[0] && pz >= zs && pz < ze) __builtin_nontemporal_store(r, p.out1 + pz * plane + col[0]);
            }
        }
        __syncthreads();
        // stage B: u^{n+2} at plane qz = pz - M on the core point
        const int qz = pz - M;
        if (qz >= zs && gin[0]) {
            const float* rq = ring[(qz - zs + 2 * M) % (M + 1)];
            const float L = cross_sum_w<M, G::EW>(rq, u1, gy[0] - y0 + M, gx[0] - x0 + M, p.w);
            bool inband;
            const float e = damp_tb(p.sp, gx[0], gy[0], qz, p.nx, p.ny, p.nz, inband);
            const float r = leap(u1[M], un[0][0], vqc, L, inband, e, qz * plane + col[0] == p.src, qs2);
            __builtin_nontemporal_store(r, p.out2 + qz * plane + col[0]);
        }
#pragma unroll
        for (int k = 0; k < NPT; ++k)
#pragma unroll
            for (int i = 0; i < 2 * M; ++i) un[k][i] = un[k][i + 1];
#pragma unroll
        for (int i = 0; i < 2 * M; ++i) u1[i] = u1[i + 1];
        buf ^= 1;
    }
}

template <int M>
void run_tb(const Tb3Args& a, hipStream_t s) {
    hipLaunchKernelGGL((k_fwd3d_cross_tb<M>), dim3(a.ntiles), dim3(kBlock3), 0, s, a);
}

}  // namespace

bool have_fwd3d_tb(int shape, int M, int rows) { return shape == SH_CROSS && M >= 1 && M <= 4 && rows == 1; }

bool launch_fwd3d_tb(const Tb3Args& a, int shape, int M, int rows, hipStream_t s) {
    if (!have_fwd3d_tb(shape, M, rows)) return false;
    switch (M) {
        case 1: run_tb<1>(a, s); return true;
        case 2: run_tb<2>(a, s); return true;
        case 3: run_tb<3>(a, s); return true;
        case 4: run_tb<4>(a, s); return true;
    }
    return false;
}

}  // namespace fdw
