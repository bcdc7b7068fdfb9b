// 3D forward and adjoint steps.
//
// Same update as the 2D kernels (Sec. 3.1-3.2, the 3D extension noted at the
// end of Sec. 3.1), on [nz][ny][nx] windows.  A block of kWaves3 waves owns a
// 64 (x) by kWaves3*RY (y) column of the grid and marches along z through
// `zchunk` planes:
//
//  * cross stencils keep the 2M+1 values of u along z for each of the thread's
//    RY points in registers (a queue rotated by renaming) and stage only the
//    current xy plane, with an M-cell halo, in LDS for the x/y neighbours;
//  * the rhombus (L1 ball) kernel tiles 64 x 4W points with four points per
//    thread and keeps only the current plane in LDS, scattering each plane's
//    in-plane sums into partial sums of the outputs it reaches (see the
//    section of that kernel);
//  * square (cube) stencils, and rhombi on very large planes, keep a ring of
//    2M+1 xy planes with halo in LDS.
//
// Every value of u^n is read from HBM once per block (plus the z warm-up of 2M
// planes per chunk and the xy halo, which neighbouring blocks of the same XCD
// also read, mostly from L2).  The forward steps advance the difference-form
// state (u^n, d^n) (see delta_update): 20 B per update (read u^n, d^n, v;
// write d^{n+1}, u^{n+1}; the scheme's minimum is 16 B).  Adjoint: 28 B
// (psi^{k+1}, u^k, psi^{k+2}, v, grad read/write, psi^k write).
//
// Difference form: points are grouped by their absolute offset pattern
// (|dx|, |dy|, |dz|), each group shares one orbit weight, and
//     L += w * (sum_of_group - |group| * u(x)).
#include "fd_kernels.h"

#include <type_traits>

namespace fdw {

namespace {

template <int M, int RY>
struct Geo3 {
    static constexpr int LW = kTileX + 2 * M;
    static constexpr int LH = kWaves3 * RY + 2 * M;
    static constexpr int PLANE = LH * LW;
};

__device__ __forceinline__ float damp_e(const Sponge& sp, int gx, int gy, int gz, int nx, int ny,
                                        int nz, bool& inband) {
    if (sp.nb <= 0) {
        inband = false;
        return 0.f;
    }
    const int dx = band_depth(gx, nx, sp.nb), dy = band_depth(gy, ny, sp.nb),
              dz = band_depth(gz, nz, sp.nb);
    inband = (dx | dy | dz) != 0;
    if (!inband) return 0.f;
    const float rx = dx * sp.inv_nb, ry = dy * sp.inv_nb, rz = dz * sp.inv_nb;
    return sp.escale * fmaf(rx, rx, fmaf(ry, ry, rz * rz));
}

// Halo of plane z of field f (interior cells excluded), zeros off the grid,
// in two halves so that the loads of the next plane can be in flight while
// the current plane is computed: fetch issues the global loads into
// registers, store writes them to LDS.  The ring is taken as the tile's 64
// columns on the M rows above and below it (thread (tx, ty) holds column tx
// at ring rows ty, ty + 8, ...) and the 2M side columns over every row of the
// plane, spread over the block.
template <int M, int RY>
struct Halo {
    static constexpr int LW = Geo3<M, RY>::LW, LH = Geo3<M, RY>::LH;
    static constexpr int NT = (2 * M + kWaves3 - 1) / kWaves3;   // top/bottom cells per thread
    static constexpr int NS = 2 * M * LH;                          // side-column cells
    static constexpr int NSL = (NS + kBlock3 - 1) / kBlock3;       // side cells per thread
    float top[NT];
    float side[NSL];

    // plane row of ring row q (0..2M-1): the M rows above, then the M below the tile
    __device__ __forceinline__ static int ring_row(int q) { return q < M ? q : q + kWaves3 * RY; }
    __device__ __forceinline__ static void side_pos(int i, int& r, int& c) {
        r = i / (2 * M);
        const int h = i - r * (2 * M);
        c = h < M ? h : kTileX + h;
    }
    __device__ __forceinline__ void fetch(const float* __restrict__ f, int nx, int ny, int nz, int x0,
                                          int y0, int z) {
        const bool zok = (unsigned)z < (unsigned)nz;
        const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;
        const int gx = x0 + tx;
        const bool xok = zok && gx < nx;
#pragma unroll
        for (int k = 0; k < NT; ++k) {
            const int q = ty + kWaves3 * k;
            const int gy = y0 - M + ring_row(q);
            top[k] = 0.f;
            if ((NT * kWaves3 == 2 * M || q < 2 * M) && xok && (unsigned)gy < (unsigned)ny)
                top[k] = f[((long long)z * ny + gy) * nx + gx];
        }
#pragma unroll
        for (int k = 0; k < NSL; ++k) {
            const int i = threadIdx.x + k * kBlock3;
            int r, c;
            side_pos(i, r, c);
            const int gy = y0 - M + r, hx = x0 - M + c;
            side[k] = 0.f;
            if ((NSL * kBlock3 == NS || i < NS) && zok && (unsigned)gy < (unsigned)ny && (unsigned)hx < (unsigned)nx)
                side[k] = f[((long long)z * ny + gy) * nx + hx];
        }
    }
    __device__ __forceinline__ void store(float* tile) const {
        const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;
#pragma unroll
        for (int k = 0; k < NT; ++k) {
            const int q = ty + kWaves3 * k;
            if (NT * kWaves3 == 2 * M || q < 2 * M) tile[ring_row(q) * LW + M + tx] = top[k];
        }
#pragma unroll
        for (int k = 0; k < NSL; ++k) {
            const int i = threadIdx.x + k * kBlock3;
            int r, c;
            side_pos(i, r, c);
            if (NSL * kBlock3 == NS || i < NS) tile[r * LW + c] = side[k];
        }
    }
};

template <int M, int RY>
__device__ __forceinline__ void load_halo(float* tile, const float* __restrict__ f, int nx, int ny,
                                          int nz, int x0, int y0, int z) {
    Halo<M, RY> h;
    h.fetch(f, nx, ny, nz, x0, y0, z);
    h.store(tile);
}

// Whole plane z (interior and halo) of field f.
template <int M, int RY>
__device__ __forceinline__ void load_plane(float* tile, const float* __restrict__ f, int nx, int ny,
                                           int nz, int x0, int y0, int z) {
    using G = Geo3<M, RY>;
    constexpr int NL = (G::PLANE + kBlock3 - 1) / kBlock3;
    const bool zok = (unsigned)z < (unsigned)nz;
    float val[NL];
#pragma unroll
    for (int k = 0; k < NL; ++k) {
        const int i = threadIdx.x + k * kBlock3;
        const int r = i / G::LW, c = i - r * G::LW;
        const int gy = y0 - M + r, gx = x0 - M + c;
        val[k] = 0.f;
        if (i < G::PLANE && zok && (unsigned)gy < (unsigned)ny && (unsigned)gx < (unsigned)nx)
            val[k] = f[((long long)z * ny + gy) * nx + gx];
    }
#pragma unroll
    for (int k = 0; k < NL; ++k) {
        const int i = threadIdx.x + k * kBlock3;
        if (i < G::PLANE) tile[i] = val[k];
    }
}

struct Pos3 {
    int tx, ty, x0, y0, zs, ze, gx;
};

template <int RY>
__device__ __forceinline__ Pos3 block_pos(int ntiles, int tiles_x, int tiles_y, int zchunk, int nz) {
    Pos3 q;
    q.tx = threadIdx.x & 63;
    q.ty = threadIdx.x >> 6;
    const int t = xcd_tile(blockIdx.x, ntiles);
    const int bx = t % tiles_x, t2 = t / tiles_x;
    const int by = t2 % tiles_y, bz = t2 / tiles_y;
    q.x0 = bx * kTileX;
    q.y0 = by * kWaves3 * RY;
    q.zs = bz * zchunk;
    q.ze = min(q.zs + zchunk, nz);
    q.gx = q.x0 + q.tx;
    return q;
}

// Byte offset b (< 2^32) from a block-uniform base pointer: the address form
// of global loads with a scalar base and a 32-bit vector offset.
__device__ __forceinline__ const float* at_b(const float* base, unsigned b) {
    return (const float*)((const char*)base + b);
}
__device__ __forceinline__ float* at_b(float* base, unsigned b) { return (float*)((char*)base + b); }

// Raw buffer access to one plane of a field: a resource over bytes
// [0, nbytes) of the plane.  The hardware range check turns an access at or
// beyond nbytes into a load of 0 or a dropped store, so a lane off the grid
// (offset kOffGrid) or a plane off the grid (nbytes = 0) costs no branch and
// no memory traffic.  Plane sizes stay below 2^31 bytes (ball_fits).
constexpr unsigned kOffGrid = 0x80000000u;
constexpr int kRsrcWord3 = 0x00020000;   // descriptor word 3: 32-bit data format
constexpr int kNonTemporal = 2;          // cache-policy bits of a streaming access
using Rsrc = __amdgpu_buffer_rsrc_t;
__device__ __forceinline__ Rsrc plane_rsrc(const float* base, unsigned nbytes) {
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<float*>(base), (short)0, (int)nbytes, kRsrcWord3);
}
// the same from a byte address held as an integer (running plane addresses
// may step outside the field; with nbytes = 0 they are never dereferenced)
__device__ __forceinline__ Rsrc plane_rsrc_at(unsigned long long addr, unsigned nbytes) {
    return __builtin_amdgcn_make_buffer_rsrc((void*)addr, (short)0, (int)nbytes, kRsrcWord3);
}
template <int AUX = 0>
__device__ __forceinline__ float bload(Rsrc r, unsigned off) {
    return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, (int)off, 0, AUX));
}
__device__ __forceinline__ void bstore_nt(float x, Rsrc r, unsigned off) {
    __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned, x), r, (int)off, 0, kNonTemporal);
}

// Halo ring of a plane for the buffer-addressed kernels (same cells and LDS
// positions as Halo), with each thread's in-plane byte offsets (kOffGrid off the grid)
// taken once: per plane only the block-uniform buffer resource changes.
template <int M, int RY>
struct PlaneHalo {
    using H = Halo<M, RY>;
    static constexpr int NT = H::NT, NS = H::NS, NSL = H::NSL, LW = H::LW;
    unsigned toff[NT], soff[NSL];
    int tlds[NT], slds[NSL];
    float top[NT], side[NSL];
    __device__ __forceinline__ void init(int nx, int ny, int x0, int y0) {
        const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;
        const int gx = x0 + tx;
#pragma unroll
        for (int k = 0; k < NT; ++k) {
            const int q = ty + kWaves3 * k;
            const int r = H::ring_row(q), gy = y0 - M + r;
            const bool ok = (NT * kWaves3 == 2 * M || q < 2 * M) && gx < nx && (unsigned)gy < (unsigned)ny;
            toff[k] = ok ? 4u * (unsigned)(gy * nx + gx) : kOffGrid;
            tlds[k] = r * LW + M + tx;
        }
#pragma unroll
        for (int k = 0; k < NSL; ++k) {
            const int i = threadIdx.x + k * kBlock3;
            int r, c;
            H::side_pos(i, r, c);
            const int gy = y0 - M + r, hx = x0 - M + c;
            const bool in = NSL * kBlock3 == NS || i < NS;
            const bool ok = in && (unsigned)gy < (unsigned)ny && (unsigned)hx < (unsigned)nx;
            soff[k] = ok ? 4u * (unsigned)(gy * nx + hx) : kOffGrid;
            slds[k] = in ? r * LW + c : -1;
        }
    }
    __device__ __forceinline__ void fetch(Rsrc plane) {
#pragma unroll
        for (int k = 0; k < NT; ++k) top[k] = bload(plane, toff[k]);
#pragma unroll
        for (int k = 0; k < NSL; ++k) side[k] = bload(plane, soff[k]);
    }
    __device__ __forceinline__ void store(float* tile) const {
#pragma unroll
        for (int k = 0; k < NT; ++k)
            if (NT * kWaves3 == 2 * M || (int)(threadIdx.x >> 6) + kWaves3 * k < 2 * M) tile[tlds[k]] = top[k];
#pragma unroll
        for (int k = 0; k < NSL; ++k)
            if (NSL * kBlock3 == NS || slds[k] >= 0) tile[slds[k]] = side[k];
    }
};

// Calls fn(integral_constant<K>, z + K) for K = 0 .. P - 1 while z + K < ze
// (K = 0 always): one period of a z loop unrolled so that register queue
// slots are compile-time constants.
template <int K, int P, class Fn>
__device__ __forceinline__ void run_phases(Fn& fn, int z, int ze) {
    if constexpr (K < P) {
        if (K == 0 || z + K < ze) {
            fn(std::integral_constant<int, K>{}, z + K);
            run_phases<K + 1, P>(fn, z, ze);
        }
    }
}


// ---------------------------------------------------------------------------
// cross: z neighbours from a register queue, x/y neighbours from LDS
// ---------------------------------------------------------------------------
template <int M, int RY>
__device__ __forceinline__ float cross_sum(const float* tile, const float* q, int row, int col,
                                           const Weights& W) {
    using G = Geo3<M, RY>;
    const float u = q[M];
    float acc = 0.f;
#pragma unroll
    for (int m = 1; m <= M; ++m) {
        const float s = (tile[row * G::LW + col - m] + tile[row * G::LW + col + m]) +
                        (tile[(row - m) * G::LW + col] + tile[(row + m) * G::LW + col]) +
                        (q[M - m] + q[M + m]);
        acc = fmaf(W.w[m], fmaf(-6.f, u, s), acc);
    }
    return acc;
}

// Sum of the cross with the z queue slot of plane z' at (z' - z0) mod P
// (PH = (z - z0) mod P); the same operations in the same order as cross_sum.
template <int M, int RY, int PH, int P>
__device__ __forceinline__ float cross_sum_q(const float* tile, const float (&q)[P], int row, int col,
                                             const Weights& W) {
    using G = Geo3<M, RY>;
    const float u = q[PH];
    float acc = 0.f;
#pragma unroll
    for (int m = 1; m <= M; ++m) {
        const float s = (tile[row * G::LW + col - m] + tile[row * G::LW + col + m]) +
                        (tile[(row - m) * G::LW + col] + tile[(row + m) * G::LW + col]) +
                        (q[(PH + P - m) % P] + q[(PH + m) % P]);
        acc = fmaf(W.w[m], fmaf(-6.f, u, s), acc);
    }
    return acc;
}

// Operands of plane z+1 (queue front u(z+1+M), d, v and the halo of u(z+1))
// are fetched while plane z is computed; the xy plane alternates between two
// LDS buffers, so one barrier per plane suffices (a buffer is rewritten only
// after every thread has passed the barrier of the plane in between).  The
// z loop is unrolled by the queue period P = 2M + 1 (queue slots rotate by
// renaming); fields are read and written through range-checked buffer
// descriptors of one plane each, whose base advances by a plane per
// iteration, so lanes and planes off the grid cost no branch.
template <int M, int RY>
__global__ __launch_bounds__(kBlock3) __attribute__((amdgpu_waves_per_eu(RY < 4 ? 4 : 2))) void k_fwd3d_cross(StepArgs p) {
    using G = Geo3<M, RY>;
    constexpr int P = 2 * M + 1;
    __shared__ float tiles[2][G::PLANE];
    if (p.trace_out) {
        for (int r = blockIdx.x * kBlock3 + threadIdx.x; r < p.nrec; r += gridDim.x * kBlock3) {
            const long long i = p.rec_lin[r];
            p.trace_out[r] = i >= 0 ? p.ucur[i] : 0.f;
        }
    }
    const Pos3 b = block_pos<RY>(p.ntiles, p.tiles_x, p.tiles_y, p.zchunk, p.nz);
    const bool xok = b.gx < p.nx;
    const long long plane = (long long)p.nx * p.ny;
    const unsigned pbytes = 4u * (unsigned)plane, vbytes = 4u * (unsigned)p.ldv_z;
    const int z0 = b.zs;
    float q[RY][P];   // u(z') at (z' - z0) mod P
    bool srccol[RY];
    unsigned coff[RY], voff[RY];
    float ry[RY];
    int dyb[RY];
    const int nb = p.sp.nb;
    const int dxb = nb > 0 ? band_depth(b.gx, p.nx, nb) : 0;
    const float rx = dxb * p.sp.inv_nb;
    const int src_z = p.src >= 0 ? (int)(p.src / plane) : -1;
    const long long src_xy = p.src >= 0 ? p.src - (long long)src_z * plane : -1;
#pragma unroll
    for (int j = 0; j < RY; ++j) {
        const int gy = b.y0 + b.ty * RY + j;
        const bool ok = xok && gy < p.ny;
        coff[j] = ok ? 4u * (unsigned)(gy * p.nx + b.gx) : kOffGrid;
        voff[j] = ok ? 4u * (unsigned)(gy * (int)p.ldv_y + b.gx) : kOffGrid;
        srccol[j] = ok && (long long)gy * p.nx + b.gx == src_xy;
        dyb[j] = (nb > 0 && ok) ? band_depth(gy, p.ny, nb) : 0;
        ry[j] = dyb[j] * p.sp.inv_nb;
    }
    // u(z0 - M .. z0 + M - 1) at (k mod P)
#pragma unroll
    for (int k = -M; k < M; ++k) {
        const int z = z0 + k;
        const bool in = (unsigned)z < (unsigned)p.nz;
        const Rsrc r = plane_rsrc(p.ucur + (in ? z : 0) * plane, in ? pbytes : 0u);
#pragma unroll
        for (int j = 0; j < RY; ++j) q[j][(k + P) % P] = bload(r, coff[j]);
    }
    PlaneHalo<M, RY> halo;
    halo.init(p.nx, p.ny, b.x0, b.y0);
    float front[RY], dd[RY], vv[RY];
    // byte addresses of u(z + M), u(z) (halo), d(z), v(z) for the next fetch
    // and of d/u^{n+1}(z) for the next update, advanced by one plane per call
    const unsigned long long pstep = 4ull * (unsigned long long)plane, vstep = 4ull * (unsigned long long)p.ldv_z;
    unsigned long long au = (unsigned long long)p.ucur + (unsigned long long)(long long)(z0 + M) * pstep;
    unsigned long long ah = (unsigned long long)p.ucur + (unsigned long long)(long long)z0 * pstep;
    unsigned long long ad = (unsigned long long)p.dcur + (unsigned long long)(long long)z0 * pstep;
    unsigned long long av = (unsigned long long)p.v + (unsigned long long)(long long)z0 * vstep;
    unsigned long long adn = (unsigned long long)p.dnext + (unsigned long long)(long long)z0 * pstep;
    unsigned long long aun = (unsigned long long)p.unext + (unsigned long long)(long long)z0 * pstep;
    auto fetch = [&](int z) {   // operands of iteration z (z < ze <= nz)
        const Rsrc ru = plane_rsrc_at(au, z + M < p.nz ? pbytes : 0u);
        const Rsrc rh = plane_rsrc_at(ah, pbytes);
        const Rsrc rd = plane_rsrc_at(ad, pbytes);
        const Rsrc rv = plane_rsrc_at(av, vbytes);
        au += pstep;
        ah += pstep;
        ad += pstep;
        av += vstep;
#pragma unroll
        for (int j = 0; j < RY; ++j) {
            front[j] = bload(ru, coff[j]);
            dd[j] = bload<kNonTemporal>(rd, coff[j]);
            vv[j] = bload<kNonTemporal>(rv, voff[j]);
        }
        halo.fetch(rh);
    };
    fetch(z0);
    const float qs = p.src >= 0 ? p.q * p.wavelet[p.step] : 0.f;
    int buf = 0;
    auto body = [&](auto ph, int z) {
        constexpr int PH = decltype(ph)::value;
        float* tile = tiles[buf];
        float ddc[RY], vvc[RY];
#pragma unroll
        for (int j = 0; j < RY; ++j) {
            q[j][(PH + M) % P] = front[j];
            ddc[j] = dd[j];
            vvc[j] = vv[j];
            tile[(b.ty * RY + j + M) * G::LW + b.tx + M] = q[j][PH];
        }
        halo.store(tile);
        if (z + 1 < b.ze) fetch(z + 1);
        __syncthreads();
        const int dzb = nb > 0 ? band_depth(z, p.nz, nb) : 0;
        const float rz = dzb * p.sp.inv_nb;
        const Rsrc rdn = plane_rsrc_at(adn, pbytes);
        const Rsrc run = plane_rsrc_at(aun, pbytes);
        adn += pstep;
        aun += pstep;
#pragma unroll
        for (int j = 0; j < RY; ++j) {
            const float L = cross_sum_q<M, RY, PH, P>(tile, q[j], b.ty * RY + j + M, b.tx + M, p.w);
            const bool inband = (dxb | dyb[j] | dzb) != 0;
            const float e = inband ? p.sp.escale * fmaf(rx, rx, fmaf(ry[j], ry[j], rz * rz)) : 0.f;
            const float d = delta_update(ddc[j], vvc[j], L, inband, e, srccol[j] && z == src_z, qs);
            bstore_nt(d, rdn, coff[j]);         // lanes off the grid: dropped
            bstore_nt(q[j][PH] + d, run, coff[j]);
        }
        buf ^= 1;
    };
    for (int z = z0; z < b.ze; z += P) run_phases<0, P>(body, z, b.ze);
}

// The same step with 64-bit addressing, for windows whose planes exceed the
// 2^31-byte range of a buffer descriptor.
template <int M, int RY>
__global__ __launch_bounds__(kBlock3) void k_fwd3d_cross_wide(StepArgs p) {
    using G = Geo3<M, RY>;
    constexpr int NQ = 2 * M + 1;
    __shared__ float tiles[2][G::PLANE];
    if (p.trace_out) {
        for (int r = blockIdx.x * kBlock3 + threadIdx.x; r < p.nrec; r += gridDim.x * kBlock3) {
            const long long i = p.rec_lin[r];
            p.trace_out[r] = i >= 0 ? p.ucur[i] : 0.f;
        }
    }
    const Pos3 b = block_pos<RY>(p.ntiles, p.tiles_x, p.tiles_y, p.zchunk, p.nz);
    const bool xok = b.gx < p.nx;
    const long long plane = (long long)p.nx * p.ny;
    float q[RY][NQ];
    bool ok[RY];
    long long col[RY], vcol[RY];   // offsets of (x, y_j) within a window / model plane
#pragma unroll
    for (int j = 0; j < RY; ++j) {
        const int gy = b.y0 + b.ty * RY + j;
        ok[j] = xok && gy < p.ny;
        col[j] = (long long)gy * p.nx + b.gx;
        vcol[j] = (long long)gy * p.ldv_y + b.gx;
#pragma unroll
        for (int i = 0; i < 2 * M; ++i) {
            const int z = b.zs - M + i;
            q[j][i] = (ok[j] && (unsigned)z < (unsigned)p.nz) ? p.ucur[z * plane + col[j]] : 0.f;
        }
    }
    Halo<M, RY> halo;
    float front[RY], dd[RY], vv[RY];
    auto fetch = [&](int z) {
#pragma unroll
        for (int j = 0; j < RY; ++j) {
            const int zz = z + M;
            const bool in = ok[j] && z < b.ze;
            front[j] = (in && zz < p.nz) ? p.ucur[zz * plane + col[j]] : 0.f;
            dd[j] = in ? __builtin_nontemporal_load(p.dcur + z * plane + col[j]) : 0.f;
            vv[j] = in ? __builtin_nontemporal_load(p.v + (long long)z * p.ldv_z + vcol[j]) : 0.f;
        }
        if (z < b.ze) halo.fetch(p.ucur, p.nx, p.ny, p.nz, b.x0, b.y0, z);
    };
    fetch(b.zs);
    int buf = 0;
    for (int z = b.zs; z < b.ze; ++z) {
        float* tile = tiles[buf];
        float ddc[RY], vvc[RY];
#pragma unroll
        for (int j = 0; j < RY; ++j) {
            q[j][2 * M] = front[j];
            ddc[j] = dd[j];
            vvc[j] = vv[j];
            tile[(b.ty * RY + j + M) * G::LW + b.tx + M] = q[j][M];
        }
        halo.store(tile);
        fetch(z + 1);
        __syncthreads();
#pragma unroll
        for (int j = 0; j < RY; ++j) {
            const float L = cross_sum<M, RY>(tile, q[j], b.ty * RY + j + M, b.tx + M, p.w);
            if (ok[j]) {
                const int gy = b.y0 + b.ty * RY + j;
                const long long k = z * plane + col[j];
                bool inband;
                const float e = damp_e(p.sp, b.gx, gy, z, p.nx, p.ny, p.nz, inband);
                const float d = delta_update(ddc[j], vvc[j], L, inband, e, k == p.src, p.q * p.wavelet[p.step]);
                __builtin_nontemporal_store(d, p.dnext + k);
                __builtin_nontemporal_store(q[j][M] + d, p.unext + k);
            }
        }
#pragma unroll
        for (int j = 0; j < RY; ++j)
#pragma unroll
            for (int i = 0; i < 2 * M; ++i) q[j][i] = q[j][i + 1];
        buf ^= 1;
    }
}

// Adjoint step and gradient term (cross), laid out like k_fwd3d_cross: the
// operands of plane z+1 (queue fronts of psi^{k+1} and u^k, psi^{k+2}, v,
// the gradient and both halos) are fetched while plane z is computed; both
// xy planes alternate between two LDS buffers (one barrier per plane); the
// z loop is unrolled by the queue period 2M + 1 and every field goes through
// range-checked per-plane buffer descriptors (a field the call does not use
// gets size 0: its loads return 0 and cost no traffic).  psi^{k+2}, v and
// the gradient are touched once per step and streamed non-temporally;
// psi^{k+1} and u^k stay cacheable for the neighbouring blocks' halo reads.
// psi^k may overwrite psi^{k+2} in place: every point is read (fetch of its
// plane) before the same thread writes it; likewise the gradient.
template <int M, int RY>
__global__ __launch_bounds__(kBlock3) __attribute__((amdgpu_waves_per_eu((RY == 1 || (RY == 2 && M <= 5)) ? 4 : 2))) void k_adj3d_cross(AdjArgs p) {
    using G = Geo3<M, RY>;
    constexpr int P = 2 * M + 1;
    __shared__ float tp[2][G::PLANE];
    __shared__ float tu[2][G::PLANE];
    const Pos3 b = block_pos<RY>(p.ntiles, p.tiles_x, p.tiles_y, p.zchunk, p.nz);
    const bool xok = b.gx < p.nx;
    const long long plane = (long long)p.nx * p.ny;
    const bool wg = p.with_grad, wu = p.with_update;
    const unsigned pbytes = 4u * (unsigned)plane, vbytes = 4u * (unsigned)p.ldv_z;
    const unsigned ubytes = wg ? pbytes : 0u, gbytes = wg ? vbytes : 0u, ppbytes = wu ? pbytes : 0u;
    const int z0 = b.zs;
    float qp[RY][P], qu[RY][P];   // psi^{k+1}(z'), u^k(z') at (z' - z0) mod P
    unsigned coff[RY], voff[RY];
    int dyb[RY];
    const int nb = p.sp.nb;
    const int dxb = nb > 0 ? band_depth(b.gx, p.nx, nb) : 0;
#pragma unroll
    for (int j = 0; j < RY; ++j) {
        const int gy = b.y0 + b.ty * RY + j;
        const bool ok = xok && gy < p.ny;
        coff[j] = ok ? 4u * (unsigned)(gy * p.nx + b.gx) : kOffGrid;
        voff[j] = ok ? 4u * (unsigned)(gy * (int)p.ldv_y + b.gx) : kOffGrid;
        dyb[j] = (nb > 0 && ok) ? band_depth(gy, p.ny, nb) : 0;
    }
#pragma unroll
    for (int k = -M; k < M; ++k) {
        const int z = z0 + k;
        const bool in = (unsigned)z < (unsigned)p.nz;
        const Rsrc rp = plane_rsrc(p.pcur + (in ? z : 0) * plane, in ? pbytes : 0u);
        const Rsrc ru = plane_rsrc(p.ufwd + (in ? z : 0) * plane, in ? ubytes : 0u);
#pragma unroll
        for (int j = 0; j < RY; ++j) {
            qp[j][(k + P) % P] = bload(rp, coff[j]);
            qu[j][(k + P) % P] = bload(ru, coff[j]);
        }
    }
    PlaneHalo<M, RY> hp, hu;
    hp.init(p.nx, p.ny, b.x0, b.y0);
    hu.init(p.nx, p.ny, b.x0, b.y0);
    float fp[RY], fu[RY], pp[RY], vv[RY], gg[RY];
    // running byte addresses: queue fronts (z + M), halo planes (z), psi^{k+2},
    // v and the gradient of the next fetch; psi^k and the gradient of the next
    // update
    const unsigned long long pstep = 4ull * (unsigned long long)plane, vstep = 4ull * (unsigned long long)p.ldv_z;
    unsigned long long apf = (unsigned long long)p.pcur + (unsigned long long)(long long)(z0 + M) * pstep;
    unsigned long long auf = (unsigned long long)p.ufwd + (unsigned long long)(long long)(z0 + M) * pstep;
    unsigned long long aph = (unsigned long long)p.pcur + (unsigned long long)(long long)z0 * pstep;
    unsigned long long auh = (unsigned long long)p.ufwd + (unsigned long long)(long long)z0 * pstep;
    unsigned long long app = (unsigned long long)p.pprev + (unsigned long long)(long long)z0 * pstep;
    unsigned long long av = (unsigned long long)p.v + (unsigned long long)(long long)z0 * vstep;
    unsigned long long ag = (unsigned long long)p.grad + (unsigned long long)(long long)z0 * vstep;
    unsigned long long apn = (unsigned long long)p.pnext + (unsigned long long)(long long)z0 * pstep;
    unsigned long long agw = ag;
    auto fetch = [&](int z) {   // operands of iteration z (z < ze <= nz)
        const bool fin = z + M < p.nz;
        const Rsrc rpf = plane_rsrc_at(apf, fin ? pbytes : 0u), ruf = plane_rsrc_at(auf, fin ? ubytes : 0u);
        const Rsrc rph = plane_rsrc_at(aph, pbytes), ruh = plane_rsrc_at(auh, ubytes);
        const Rsrc rpp = plane_rsrc_at(app, ppbytes), rv = plane_rsrc_at(av, vbytes), rg = plane_rsrc_at(ag, gbytes);
        apf += pstep;
        auf += pstep;
        aph += pstep;
        auh += pstep;
        app += pstep;
        av += vstep;
        ag += vstep;
#pragma unroll
        for (int j = 0; j < RY; ++j) {
            fp[j] = bload(rpf, coff[j]);
            fu[j] = bload(ruf, coff[j]);
            pp[j] = bload<kNonTemporal>(rpp, coff[j]);
            vv[j] = bload<kNonTemporal>(rv, voff[j]);
            gg[j] = bload<kNonTemporal>(rg, voff[j]);
        }
        hp.fetch(rph);
        if (wg) hu.fetch(ruh);
    };
    fetch(z0);
    int buf = 0;
    auto body = [&](auto ph, int z) {
        constexpr int PH = decltype(ph)::value;
        float* tpb = tp[buf];
        float* tub = tu[buf];
        float ppc[RY], vvc[RY], ggc[RY];
#pragma unroll
        for (int j = 0; j < RY; ++j) {
            qp[j][(PH + M) % P] = fp[j];
            qu[j][(PH + M) % P] = fu[j];
            ppc[j] = pp[j];
            vvc[j] = vv[j];
            ggc[j] = gg[j];
            tpb[(b.ty * RY + j + M) * G::LW + b.tx + M] = qp[j][PH];
            tub[(b.ty * RY + j + M) * G::LW + b.tx + M] = qu[j][PH];
        }
        hp.store(tpb);
        if (wg) hu.store(tub);
        if (z + 1 < b.ze) fetch(z + 1);
        __syncthreads();
        const int dzb = nb > 0 ? band_depth(z, p.nz, nb) : 0;
        const Rsrc rg = plane_rsrc_at(agw, gbytes), rn = plane_rsrc_at(apn, wu ? pbytes : 0u);
        agw += vstep;
        apn += pstep;
#pragma unroll
        for (int j = 0; j < RY; ++j) {
            const int row = b.ty * RY + j + M;
            const float pc = qp[j][PH];
            if (wg) {
                const float Lu = cross_sum_q<M, RY, PH, P>(tub, qu[j], row, b.tx + M, p.w);
                bstore_nt(fmaf(grad_factor(p.gparam, p.gscale, vvc[j]) * pc, Lu, ggc[j]), rg, voff[j]);
            }
            if (wu) {
                const float Lp = cross_sum_q<M, RY, PH, P>(tpb, qp[j], row, b.tx + M, p.w);
                const bool inband = (dxb | dyb[j] | dzb) != 0;
                float r;
                if (!inband) {
                    r = fmaf(vvc[j], Lp, 2.f * pc - ppc[j]);
                } else {
                    const float rx = dxb * p.sp.inv_nb, ry = dyb[j] * p.sp.inv_nb, rz = dzb * p.sp.inv_nb;
                    const float e = p.sp.escale * fmaf(rx, rx, fmaf(ry, ry, rz * rz));
                    r = fmaf(-(1.f - e), ppc[j], 2.f * pc);
                    r = fmaf(vvc[j], Lp, r);
                    r = r / (1.f + e);
                }
                bstore_nt(r, rn, coff[j]);
            }
        }
        buf ^= 1;
    };
    for (int z = z0; z < b.ze; z += P) run_phases<0, P>(body, z, b.ze);
}

// The same step with 64-bit addressing, for windows whose planes exceed the
// 2^31-byte range of a buffer descriptor.
template <int M, int RY>
__global__ __launch_bounds__(kBlock3) void k_adj3d_cross_wide(AdjArgs p) {
    using G = Geo3<M, RY>;
    constexpr int NQ = 2 * M + 1;
    __shared__ float tp[2][G::PLANE];
    __shared__ float tu[2][G::PLANE];
    const Pos3 b = block_pos<RY>(p.ntiles, p.tiles_x, p.tiles_y, p.zchunk, p.nz);
    const bool xok = b.gx < p.nx;
    const long long plane = (long long)p.nx * p.ny;
    const bool wg = p.with_grad, wu = p.with_update;
    float qp[RY][NQ], qu[RY][NQ];
    bool ok[RY];
    long long col[RY], vcol[RY];
#pragma unroll
    for (int j = 0; j < RY; ++j) {
        const int gy = b.y0 + b.ty * RY + j;
        ok[j] = xok && gy < p.ny;
        col[j] = (long long)gy * p.nx + b.gx;
        vcol[j] = (long long)gy * p.ldv_y + b.gx;
#pragma unroll
        for (int i = 0; i < 2 * M; ++i) {
            const int z = b.zs - M + i;
            const bool in = ok[j] && (unsigned)z < (unsigned)p.nz;
            qp[j][i] = in ? p.pcur[z * plane + col[j]] : 0.f;
            qu[j][i] = (in && wg) ? p.ufwd[z * plane + col[j]] : 0.f;
        }
    }
    Halo<M, RY> hp, hu;
    float fp[RY], fu[RY], pp[RY], vv[RY], gg[RY];
    auto fetch = [&](int z) {
#pragma unroll
        for (int j = 0; j < RY; ++j) {
            const int zz = z + M;
            const bool in = ok[j] && z < b.ze;
            const bool fin = in && zz < p.nz;
            fp[j] = fin ? p.pcur[zz * plane + col[j]] : 0.f;
            fu[j] = (fin && wg) ? p.ufwd[zz * plane + col[j]] : 0.f;
            pp[j] = (in && wu) ? __builtin_nontemporal_load(p.pprev + z * plane + col[j]) : 0.f;
            vv[j] = in ? __builtin_nontemporal_load(p.v + (long long)z * p.ldv_z + vcol[j]) : 0.f;
            gg[j] = (in && wg) ? __builtin_nontemporal_load(p.grad + (long long)z * p.ldv_z + vcol[j]) : 0.f;
        }
        if (z < b.ze) {
            hp.fetch(p.pcur, p.nx, p.ny, p.nz, b.x0, b.y0, z);
            if (wg) hu.fetch(p.ufwd, p.nx, p.ny, p.nz, b.x0, b.y0, z);
        }
    };
    fetch(b.zs);
    int buf = 0;
    for (int z = b.zs; z < b.ze; ++z) {
        float* tpb = tp[buf];
        float* tub = tu[buf];
        float ppc[RY], vvc[RY], ggc[RY];
#pragma unroll
        for (int j = 0; j < RY; ++j) {
            qp[j][2 * M] = fp[j];
            qu[j][2 * M] = fu[j];
            ppc[j] = pp[j];
            vvc[j] = vv[j];
            ggc[j] = gg[j];
            tpb[(b.ty * RY + j + M) * G::LW + b.tx + M] = qp[j][M];
            tub[(b.ty * RY + j + M) * G::LW + b.tx + M] = qu[j][M];
        }
        hp.store(tpb);
        if (wg) hu.store(tub);
        fetch(z + 1);
        __syncthreads();
#pragma unroll
        for (int j = 0; j < RY; ++j) {
            const int row = b.ty * RY + j + M;
            const float Lp = cross_sum<M, RY>(tpb, qp[j], row, b.tx + M, p.w);
            const float Lu = wg ? cross_sum<M, RY>(tub, qu[j], row, b.tx + M, p.w) : 0.f;
            if (ok[j]) {
                const int gy = b.y0 + b.ty * RY + j;
                const long long k = z * plane + col[j];
                const long long kv = (long long)z * p.ldv_z + vcol[j];
                const float pc = qp[j][M];
                if (wg)
                    __builtin_nontemporal_store(fmaf(grad_factor(p.gparam, p.gscale, vvc[j]) * pc, Lu, ggc[j]),
                                                p.grad + kv);
                if (wu) {
                    bool inband;
                    const float e = damp_e(p.sp, b.gx, gy, z, p.nx, p.ny, p.nz, inband);
                    float r;
                    if (!inband) {
                        r = fmaf(vvc[j], Lp, 2.f * pc - ppc[j]);
                    } else {
                        r = fmaf(-(1.f - e), ppc[j], 2.f * pc);
                        r = fmaf(vvc[j], Lp, r);
                        r = r / (1.f + e);
                    }
                    __builtin_nontemporal_store(r, p.pnext + k);
                }
            }
        }
#pragma unroll
        for (int j = 0; j < RY; ++j)
#pragma unroll
            for (int i = 0; i < 2 * M; ++i) {
                qp[j][i] = qp[j][i + 1];
                qu[j][i] = qu[j][i + 1];
            }
        buf ^= 1;
    }
}

// ---------------------------------------------------------------------------
// rhombus / square: ring of 2M+1 planes in LDS
// ---------------------------------------------------------------------------
// Sum over the group of offsets (+-DX, +-DY, +-DZ) of plane(s) at row/col.
template <int M, int RY, int DX, int DY>
__device__ __forceinline__ float inplane(const float* t, int row, int col) {
    using G = Geo3<M, RY>;
    const float* c = t + row * G::LW + col;
    if constexpr (DX == 0 && DY == 0) return c[0];
    else if constexpr (DY == 0) return c[-DX] + c[DX];
    else if constexpr (DX == 0) return c[-DY * G::LW] + c[DY * G::LW];
    else return (c[-DY * G::LW - DX] + c[-DY * G::LW + DX]) + (c[DY * G::LW - DX] + c[DY * G::LW + DX]);
}

// Groups (+-DX, +-DY, +-DZ) of one |dz| layer, DY outer, DX inner.
template <int SHAPE, int M, int RY, int DZ, int DY, int DX>
__device__ __forceinline__ void gen_xy(const float* pm, const float* p0, const float* pp, int row,
                                       int col, float u, float& acc, const Weights& W) {
    if constexpr (DY <= M) {
        if constexpr (DX > M) {
            gen_xy<SHAPE, M, RY, DZ, DY + 1, 0>(pm, p0, pp, row, col, u, acc, W);
        } else {
            constexpr int a = cmax_(DX, cmax_(DY, DZ)), c = cmin_(DX, cmin_(DY, DZ));
            constexpr int bmid = DX + DY + DZ - a - c;
            if constexpr ((DX | DY | DZ) != 0 && in_shape3(SHAPE, M, a, bmid, c)) {
                constexpr int o = orbit3(SHAPE, M, a, bmid, c);
                constexpr float cnt = (DX ? 2.f : 1.f) * (DY ? 2.f : 1.f) * (DZ ? 2.f : 1.f);
                float s;
                if constexpr (DZ == 0) s = inplane<M, RY, DX, DY>(p0, row, col);
                else s = inplane<M, RY, DX, DY>(pm, row, col) + inplane<M, RY, DX, DY>(pp, row, col);
                acc = fmaf(W.w[o], fmaf(-cnt, u, s), acc);
            }
            gen_xy<SHAPE, M, RY, DZ, DY, DX + 1>(pm, p0, pp, row, col, u, acc, W);
        }
    }
}

// Layers |dz| = DZ..M.  Plane of offset d (d in [-M, M]) sits in ring slot
// (base + d) mod NR, base = slot of the output plane.
template <int SHAPE, int M, int RY, int NR, int DZ>
__device__ __forceinline__ void gen_layers_r(const float* ring, int base, int row, int col, float u,
                                             float& acc, const Weights& W) {
    if constexpr (DZ <= M) {
        using G = Geo3<M, RY>;
        int sm = base - DZ, sp = base + DZ;
        if (sm < 0) sm += NR;
        if (sp >= NR) sp -= NR;
        gen_xy<SHAPE, M, RY, DZ, 0, 0>(ring + sm * G::PLANE, ring + base * G::PLANE,
                                       ring + sp * G::PLANE, row, col, u, acc, W);
        gen_layers_r<SHAPE, M, RY, NR, DZ + 1>(ring, base, row, col, u, acc, W);
    }
}

template <int SHAPE, int M, int RY, int DZ>
__device__ __forceinline__ void gen_layers(const float* ring, int base, int row, int col, float u,
                                           float& acc, const Weights& W) {
    gen_layers_r<SHAPE, M, RY, 2 * M + 1, DZ>(ring, base, row, col, u, acc, W);
}

template <int SHAPE, int M, int RY, int NF>
struct RingLDS {
    float f[NF][2 * M + 1][Geo3<M, RY>::PLANE];
};

// Registers holding one whole plane (interior and halo) between its global
// loads and its LDS store.  Thread (tx, ty) holds column x0 + tx at rows ty,
// ty + 8, ... (one index step of 8 rows per load, coalesced along x); the 2M
// halo columns are spread over the block.
template <int M, int RY>
struct PlaneRegs {
    static constexpr int LW = Geo3<M, RY>::LW, LH = Geo3<M, RY>::LH;
    static constexpr int NR = (LH + kWaves3 - 1) / kWaves3;   // rows per thread, main columns
    static constexpr int NH = 2 * M * LH;                      // halo cells
    static constexpr int NHL = (NH + kBlock3 - 1) / kBlock3;   // halo cells per thread
    float val[NR];
    float hv[NHL];
    __device__ __forceinline__ void fetch(const float* __restrict__ f, int nx, int ny, int nz, int x0,
                                          int y0, int z) {
        const bool zok = (unsigned)z < (unsigned)nz;
        const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;
        const int gx = x0 + tx;
        const bool xok = zok && gx < nx;
        long long idx = ((long long)z * ny + (y0 - M + ty)) * nx + gx;   // the thread's k-th row
        const long long step = (long long)kWaves3 * nx;
#pragma unroll
        for (int k = 0; k < NR; ++k) {
            const int r = ty + kWaves3 * k, gy = y0 - M + r;
            val[k] = 0.f;
            if ((NR * kWaves3 == LH || r < LH) && xok && (unsigned)gy < (unsigned)ny) val[k] = f[idx];
            idx += step;
        }
#pragma unroll
        for (int k = 0; k < NHL; ++k) {
            const int i = threadIdx.x + k * kBlock3;
            const int r = i / (2 * M), h = i - r * (2 * M);
            const int c = h < M ? h : kTileX + h;
            const int gy = y0 - M + r, hx = x0 - M + c;
            hv[k] = 0.f;
            if ((NHL * kBlock3 == NH || i < NH) && zok && (unsigned)gy < (unsigned)ny && (unsigned)hx < (unsigned)nx)
                hv[k] = f[((long long)z * ny + gy) * nx + hx];
        }
    }
    __device__ __forceinline__ void store(float* tile) const {
        const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;
#pragma unroll
        for (int k = 0; k < NR; ++k) {
            const int r = ty + kWaves3 * k;
            if (NR * kWaves3 == LH || r < LH) tile[r * LW + tx + M] = val[k];
        }
#pragma unroll
        for (int k = 0; k < NHL; ++k) {
            const int i = threadIdx.x + k * kBlock3;
            const int r = i / (2 * M), h = i - r * (2 * M);
            if (NHL * kBlock3 == NH || i < NH) tile[r * LW + (h < M ? h : kTileX + h)] = hv[k];
        }
    }
};

// Ring of 2M+2 planes: plane p lives in slot (p - zs + M) mod (2M+2).  While
// plane z is computed, plane z+M+1 goes into the slot of plane z-M-1, which
// no thread reads any more once the barrier at the top of iteration z has
// passed; so one barrier per plane suffices, and the global loads of plane
// z+M+2 are in flight during the computation.
template <int SHAPE, int M, int RY>
__global__ __launch_bounds__(kBlock3) void k_fwd3d_gen(StepArgs p) {
    using G = Geo3<M, RY>;
    constexpr int NR = 2 * M + 2;
    __shared__ float ring[NR * G::PLANE];
    if (p.trace_out) {
        for (int r = blockIdx.x * kBlock3 + threadIdx.x; r < p.nrec; r += gridDim.x * kBlock3) {
            const long long i = p.rec_lin[r];
            p.trace_out[r] = i >= 0 ? p.ucur[i] : 0.f;
        }
    }
    const Pos3 b = block_pos<RY>(p.ntiles, p.tiles_x, p.tiles_y, p.zchunk, p.nz);
    PlaneRegs<M, RY> pf;
    for (int i = 0; i < 2 * M + 1; ++i) {
        pf.fetch(p.ucur, p.nx, p.ny, p.nz, b.x0, b.y0, b.zs - M + i);
        pf.store(ring + i * G::PLANE);
    }
    float dd[RY], vv[RY];
    auto fetch_pointwise = [&](int z) {
#pragma unroll
        for (int j = 0; j < RY; ++j) {
            const int gy = b.y0 + b.ty * RY + j;
            const bool ok = b.gx < p.nx && gy < p.ny && z < b.ze;
            dd[j] = ok ? p.dcur[((long long)z * p.ny + gy) * p.nx + b.gx] : 0.f;
            vv[j] = ok ? p.v[(long long)z * p.ldv_z + (long long)gy * p.ldv_y + b.gx] : 0.f;
        }
    };
    pf.fetch(p.ucur, p.nx, p.ny, p.nz, b.x0, b.y0, b.zs + M + 1);
    fetch_pointwise(b.zs);
    int base = M;   // slot of plane z
    for (int z = b.zs; z < b.ze; ++z) {
        __syncthreads();
        int slot = base + M + 1;
        if (slot >= NR) slot -= NR;
        pf.store(ring + slot * G::PLANE);          // plane z+M+1, needed from the next plane on
        float ddc[RY], vvc[RY];
#pragma unroll
        for (int j = 0; j < RY; ++j) {
            ddc[j] = dd[j];
            vvc[j] = vv[j];
        }
        if (z + 1 < b.ze) pf.fetch(p.ucur, p.nx, p.ny, p.nz, b.x0, b.y0, z + M + 2);
        fetch_pointwise(z + 1);
#pragma unroll
        for (int j = 0; j < RY; ++j) {
            const int row = b.ty * RY + j + M, col = b.tx + M;
            const float uc = ring[base * G::PLANE + row * G::LW + col];
            float Ls = 0.f;
            gen_layers_r<SHAPE, M, RY, NR, 0>(ring, base, row, col, uc, Ls, p.w);
            const int gy = b.y0 + b.ty * RY + j;
            if (b.gx < p.nx && gy < p.ny) {
                const long long k = ((long long)z * p.ny + gy) * p.nx + b.gx;
                bool inband;
                const float e = damp_e(p.sp, b.gx, gy, z, p.nx, p.ny, p.nz, inband);
                const float d = delta_update(ddc[j], vvc[j], Ls, inband, e, k == p.src, p.q * p.wavelet[p.step]);
                p.dnext[k] = d;
                p.unext[k] = uc + d;
            }
        }
        base = base + 1 == NR ? 0 : base + 1;
    }
}

// ---------------------------------------------------------------------------
// L1 ball (3D rhombus): in-plane difference sums scattered along z
// ---------------------------------------------------------------------------
// Split each offset d = (p, dz) into its in-plane part p and dz.  The in-plane
// parts form groups (a, b), a >= b >= 0, 1 <= a + b <= M: the points
// (+-a, +-b), (+-b, +-a), n_ab of them (4 when b = 0 or a = b, else 8).  With
//     D_ab(z') = sum_{p in (a, b)} u(x + p, z') - n_ab u(x, z')
// (a small difference, formed from the LDS copy of plane z') the centre-free
// difference form of the stencil at plane o is
//     sum_ab sum_{|t| <= M-a-b} w(a,b,|t|) D_ab(o + t)
//   + sum_{m=1}^{M} wc(m) [(u(o+m) - u(o)) + (u(o-m) - u(o))],
// wc(m) = w(0,0,m) + sum_{a+b <= M-m} n_ab w(a,b,m) (formed on the host in
// FP64, rounded once): the same sum as the plain form, every term a small
// difference.  The block marches along z; when plane z' arrives (one LDS
// buffer per plane, loaded straight from memory into LDS by buffer loads
// with the LDS flag, double-buffered, one barrier per plane) every group's
// D_ab(z') is formed once and added with its weights into the partial sums
// of the outputs z' - (M-a-b) .. z' + (M-a-b), and the z differences
// u(z') - u(z'-m), m = 1..M, go to outputs z' - m and z'; output z' - M is
// then complete and updated.  Transfers whose offset fails the range check
// (cells off the grid, planes off the grid) write zeros into LDS, as the
// stencil reads them.  A thread owns four consecutive points of a row
// (16 threads per 64-point row), so a row window of its points' in-plane
// neighbours is 1 + MP/2 aligned 16-byte LDS reads (rows -R and +R are
// added column by column before their x pairs are formed, the column sums
// shared by the four points), and per point it keeps 2M partial sums and
// M queued values of u.  The z loop is unrolled by the
// period 2M, so partial sums, queue entries and the LDS buffer are
// compile-time slots.  Each z chunk runs M planes before and after its own.
__host__ __device__ constexpr int ball_ngroups(int M) {
    int n = 0;
    for (int s = 1; s <= M; ++s) n += s / 2 + 1;
    return n;
}
// index of group (a, b), a >= b: groups ordered by a + b, then b
__host__ __device__ constexpr int ball_gidx(int a, int b) {
    int g = 0;
    for (int s = 1; s < a + b; ++s) g += s / 2 + 1;
    return g + b;
}
// orbit of the offset with absolute components (x, y, z), any order
__host__ __device__ constexpr int ball_orbit(int M, int x, int y, int z) {
    return orbit3_of(SH_RHOMBUS, M, x, y, z);
}

template <int B, int E, class F>
__device__ __forceinline__ void cfor(F&& f) {
    if constexpr (B < E) {
        f(std::integral_constant<int, B>{});
        cfor<B + 1, E>(f);
    }
}

template <int M, int W>   // W waves per block
struct BallGeo {
    static constexpr int MP = (M + 3) / 4 * 4;   // x halo, whole 16-byte units
    static constexpr int TX = 64, TY = 4 * W;    // tile: 16 threads x 4 points per row, 4W rows
    static constexpr int LW = TX + 2 * MP, LH = TY + 2 * M;
    static constexpr int PLANE = LW * LH;        // floats per LDS plane
    static constexpr int NTH = 64 * W;
};

using LdsPtr = __attribute__((address_space(3))) void*;
typedef unsigned U4 __attribute__((ext_vector_type(4)));
typedef float F4 __attribute__((ext_vector_type(4)));
// (16-byte operand loads go through plain global pointers: the 128-bit raw
// buffer load builtin is narrowed to one dword by this compiler when its
// elements are bit-cast to float one by one)
__device__ __forceinline__ void bstore4_nt(U4 x, Rsrc r, unsigned off) {
    __builtin_amdgcn_raw_buffer_store_b128(x, r, (int)off, 0, kNonTemporal);
}
// 4 * UNIT bytes per lane from global memory straight into LDS at buf + lane * UNIT floats
// (the LDS address is taken from the low 32 bits of the generic address of
// an LDS location: a generic-to-LDS pointer cast here makes this compiler
// emit an invalid null-pointer test on the aperture register)
template <int UNIT>
__device__ __forceinline__ void bload_lds(Rsrc r, float* buf, unsigned off) {
    const LdsPtr dst = (LdsPtr)(uintptr_t)(unsigned)(uintptr_t)buf;
    if constexpr (UNIT == 4) __builtin_amdgcn_raw_ptr_buffer_load_lds(r, dst, 16, off, 0, 0, 0);
    else __builtin_amdgcn_raw_ptr_buffer_load_lds(r, dst, 4, off, 0, 0, 0);
}

// In-plane sums of rows -R and +R (row 0 alone for R = 0) into the group
// sums S of the thread's four points; rm and rp are the thread's first LDS
// columns of the two rows.  For R >= 1 the two rows are added column by
// column first (over the columns the rows use), then the column sums are
// paired at x distances 1 .. M - R.  The first contribution to group (a, b),
// a >= b, comes from R = b and is assigned.
template <int M, int MP, int R, int NG>
__device__ __forceinline__ void ball_row_pair(const float* rm, const float* rp, float (&S)[NG][4],
                                              float (&uc)[4]) {
    constexpr int lo = MP - (M - R), hi = MP + 3 + (M - R);
    constexpr int k0 = lo / 4, k1 = hi / 4;
    float win[4 * (k1 + 1)];
    cfor<k0, k1 + 1>([&](auto kc) {
        constexpr int k = decltype(kc)::value;
        const float4 a = reinterpret_cast<const float4*>(__builtin_assume_aligned(rm, 16))[k];
        if constexpr (R == 0) {
            win[4 * k] = a.x;
            win[4 * k + 1] = a.y;
            win[4 * k + 2] = a.z;
            win[4 * k + 3] = a.w;
        } else {
            const float4 b = reinterpret_cast<const float4*>(__builtin_assume_aligned(rp, 16))[k];
            win[4 * k] = a.x + b.x;
            win[4 * k + 1] = a.y + b.y;
            win[4 * k + 2] = a.z + b.z;
            win[4 * k + 3] = a.w + b.w;
            // each 16-byte piece summed before the next pair of reads
#pragma unroll
            for (int j = 4 * k; j < 4 * k + 4; ++j)
                if (j >= lo && j <= hi) __asm__ volatile("" : "+v"(win[j])::"memory");
        }
    });
    cfor<0, 4>([&](auto ic) {
        constexpr int i = decltype(ic)::value;
        if constexpr (R == 0) uc[i] = win[MP + i];
        else S[ball_gidx(R, 0)][i] += win[MP + i];
        cfor<1, M - R + 1>([&](auto kc) {
            constexpr int k = decltype(kc)::value;
            constexpr int a = k > R ? k : R, b = k > R ? R : k;
            constexpr int g = ball_gidx(a, b);
            const float pr = win[MP + i - k] + win[MP + i + k];
            if constexpr (b == R) S[g][i] = pr;
            else S[g][i] += pr;
        });
    });
}

// Group (A, B) is complete: D = S - n u, added into the partial sums of the
// outputs z' + t, |t| <= M - A - B (slot (PH + t) mod Q).  Its t = M - 1
// contribution (group (1, 0) only) is the first that output receives.
template <int M, int Q, int PH, int A, int B, int NG>
__device__ __forceinline__ void ball_scatter(float (&acc)[Q][4], const float (&S)[NG][4], const float (&uc)[4],
                                             const Weights& W) {
    constexpr int mz = M - A - B;
    constexpr float n = (B == 0 || A == B) ? 4.f : 8.f;
    constexpr int g = ball_gidx(A, B);
    cfor<0, 4>([&](auto ic) {
        constexpr int i = decltype(ic)::value;
        const float D = fmaf(-n, uc[i], S[g][i]);
        cfor<0, 2 * mz + 1>([&](auto tc) {
            constexpr int t = decltype(tc)::value - mz;
            constexpr int o = ball_orbit(M, A, B, t < 0 ? -t : t);
            constexpr int slot = ((PH + t) % Q + Q) % Q;
            if constexpr (A == 1 && B == 0 && t == mz) acc[slot][i] = W.w[o] * D;
            else acc[slot][i] = fmaf(W.w[o], D, acc[slot][i]);
            __asm__ volatile("" : "+v"(acc[slot][i]));   // added here, not sunk to the end
        });
    });
}

// Rows +-R, then the groups (R, b) they complete.
template <int M, int MP, int LW, int Q, int PH, int R, int NG>
__device__ __forceinline__ void ball_rows_from(const float* base, float (&S)[NG][4], float (&uc)[4],
                                               float (&acc)[Q][4], const Weights& W) {
    if constexpr (R <= M) {
        // The empty asm statements take the group sums as operands, so each
        // row is summed before the next row is read (otherwise the compiler
        // gathers every row's LDS reads at the top, all windows live at once).
        auto fence = [&]() {
#pragma unroll
            for (int g = 0; g < NG; ++g)
#pragma unroll
                for (int i = 0; i < 4; ++i) __asm__ volatile("" : "+v"(S[g][i])::"memory");
        };
        if constexpr (R == 0) {
            ball_row_pair<M, MP, 0, NG>(base, base, S, uc);
            fence();
        } else {
            ball_row_pair<M, MP, R, NG>(base - R * LW, base + R * LW, S, uc);
            fence();
            cfor<0, (R < M - R ? R : M - R) + 1>([&](auto bc) {
                ball_scatter<M, Q, PH, R, decltype(bc)::value, NG>(acc, S, uc, W);
            });
        }
        ball_rows_from<M, MP, LW, Q, PH, R + 1, NG>(base, S, uc, acc, W);
    }
}

// Window and model planes are addressed with 32-bit byte offsets below 2^31.
bool planes_fit(const StepArgs& a) {
    return (long long)a.nx * a.ny < (1LL << 29) && a.ldv_z < (1LL << 29);
}

// VEC: the window and model rows are 16-byte aligned (nx, ldv_y, ldv_z
// multiples of 4, 16-byte aligned fields): 16-byte loads and stores; else
// 4-byte ones.
template <int M, int W, int VEC>
__global__ __launch_bounds__(64 * W) __attribute__((amdgpu_waves_per_eu(M <= 2 ? 4 : 2))) void k_fwd3d_ball(StepArgs p) {
    using BG = BallGeo<M, W>;
    constexpr int MP = BG::MP, LW = BG::LW, LH = BG::LH, PLANE = BG::PLANE, NTH = BG::NTH;
    constexpr int Q = 2 * M;
    constexpr int NG = ball_ngroups(M);
    constexpr int UNIT = VEC ? 4 : 1;                  // floats per transfer
    constexpr int NF = PLANE / UNIT;                   // transfers per LDS plane
    constexpr int NPASS = (NF + NTH - 1) / NTH;
    __shared__ __attribute__((aligned(16))) float lds[2 * PLANE];
    if (p.trace_out) {
        for (int r = blockIdx.x * NTH + threadIdx.x; r < p.nrec; r += gridDim.x * NTH) {
            const long long i = p.rec_lin[r];
            p.trace_out[r] = i >= 0 ? p.ucur[i] : 0.f;
        }
    }
    const int t = xcd_tile(blockIdx.x, p.ntiles);
    const int bx = t % p.tiles_x, t2 = t / p.tiles_x;
    const int by = t2 % p.tiles_y, bz = t2 / p.tiles_y;
    const int x0 = bx * BG::TX, y0 = by * BG::TY;
    const int zs = bz * p.zchunk, ze = min(zs + p.zchunk, p.nz);
    const int tq = threadIdx.x & 15, ty = threadIdx.x >> 4;
    const int gx = x0 + 4 * tq, gy = y0 + ty;
    const long long plane = (long long)p.nx * p.ny;
    const unsigned pbytes = 4u * (unsigned)plane, vbytes = 4u * (unsigned)p.ldv_z;
    const bool yok = gy < p.ny;
    // byte offsets of the thread's points in a window plane and a model plane
    unsigned coff[VEC ? 1 : 4], voff[VEC ? 1 : 4];
#pragma unroll
    for (int i = 0; i < (VEC ? 1 : 4); ++i) {
        const bool ok = yok && gx + i < p.nx;
        coff[i] = ok ? 4u * (unsigned)(gy * p.nx + gx + i) : kOffGrid;
        voff[i] = ok ? 4u * (unsigned)(gy * (int)p.ldv_y + gx + i) : kOffGrid;
    }
    // element offsets of the first point, 0 off the grid (16-byte operand loads)
    const unsigned cidx = coff[0] == kOffGrid ? 0u : coff[0] / 4;
    const unsigned vidx = voff[0] == kOffGrid ? 0u : voff[0] / 4;
    // damping: x/y band part per point, z part per plane
    const int nb = p.sp.nb;
    const int dyb = (nb > 0 && yok) ? band_depth(gy, p.ny, nb) : 0;
    const float ry = dyb * p.sp.inv_nb;
    float exy[4];
    bool xyband[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const int dxb = nb > 0 ? band_depth(gx + i, p.nx, nb) : 0;
        const float rx = dxb * p.sp.inv_nb;
        exy[i] = fmaf(rx, rx, ry * ry);
        xyband[i] = (dxb | dyb) != 0;
    }
    const int src_z = p.src >= 0 ? (int)(p.src / plane) : -1;
    const long long src_xy = p.src >= 0 ? p.src - (long long)src_z * plane : -1;
    const long long my_xy = (long long)gy * p.nx + gx;
    const int src_i = (yok && src_xy >= my_xy && src_xy < my_xy + 4 && gx + (int)(src_xy - my_xy) < p.nx)
                          ? (int)(src_xy - my_xy) : -1;
    const float qs = p.src >= 0 ? p.q * p.wavelet[p.step] : 0.f;
    // transfers of an LDS plane: unit f of the plane (row-major, UNIT floats)
    // is loaded by thread f mod NTH in pass f / NTH
    unsigned doff[NPASS];
#pragma unroll
    for (int k = 0; k < NPASS; ++k) {
        const int f = threadIdx.x + NTH * k;
        const int row = f / (LW / UNIT), c = (f - row * (LW / UNIT)) * UNIT;
        const int yy = y0 - M + row, xx = x0 - MP + c;
        const bool ok = f < NF && (unsigned)yy < (unsigned)p.ny && (unsigned)xx < (unsigned)p.nx;
        doff[k] = ok ? 4u * (unsigned)(yy * p.nx + xx) : kOffGrid;
    }
    const int z_begin = zs - M, z_end = ze + M;
    const unsigned long long pstep = 4ull * (unsigned long long)plane, vstep = 4ull * (unsigned long long)p.ldv_z;
    // running byte addresses: next plane to load into LDS; d, v of the next
    // output to prefetch; d, u^{n+1} of the next output to finalise
    unsigned long long au = (unsigned long long)p.ucur + (unsigned long long)(long long)z_begin * pstep;
    unsigned long long ad = (unsigned long long)p.dcur + (unsigned long long)(long long)(z_begin - M) * pstep;
    unsigned long long av = (unsigned long long)p.v + (unsigned long long)(long long)(z_begin - M) * vstep;
    unsigned long long adn = (unsigned long long)p.dnext + (unsigned long long)(long long)(z_begin - M) * pstep;
    unsigned long long aun = (unsigned long long)p.unext + (unsigned long long)(long long)(z_begin - M) * pstep;
    int zload = z_begin, zdv = z_begin - M;
    auto load_plane_lds = [&](float* buf) {   // plane zload into buf, then advance
        const Rsrc r = plane_rsrc_at(au, (unsigned)zload < (unsigned)p.nz ? pbytes : 0u);
        au += pstep;
        ++zload;
#pragma unroll
        for (int k = 0; k < NPASS; ++k) {
            if (NPASS * NTH == NF || (int)threadIdx.x + NTH * k < NF)
                bload_lds<UNIT>(r, buf + ((threadIdx.x & ~63) + NTH * k) * UNIT, doff[k]);
        }
    };
    // AHEAD (M = 4, 5, where eight more registers leave the occupancy as it
    // is): d, v of an output are fetched one plane ahead, and the next plane's
    // LDS load is issued once this plane's LDS reads are done.  The compiler
    // makes every LDS read wait for LDS-flag loads still in flight, so a load
    // issued before the reads is waited for at once; issued after them, it
    // and the d, v loads have the rest of the plane's work to land.  The
    // update is then stored at once, on every plane (range-checked to nothing
    // outside the chunk), so that the wait before the next barrier can leave
    // exactly those stores in flight.
    constexpr bool AHEAD = M == 4 || M == 5;
    float dv[AHEAD ? 2 : 1][2][4];   // [slot][d, v][point]
    auto fetch_dv = [&](float (&dd)[4], float (&vv)[4]) {   // d, v of output zdv, then advance
        const bool in = zdv >= zs && zdv < ze;
        const Rsrc rd = plane_rsrc_at(ad, in ? pbytes : 0u);
        const Rsrc rv = plane_rsrc_at(av, in ? vbytes : 0u);
        ad += pstep;
        av += vstep;
        ++zdv;
        if constexpr (VEC) {
            // planes outside the chunk read plane 0 and lanes off the grid the
            // plane's first 16 bytes: loaded, never used
            const long long zo = in ? zdv - 1 : 0;
            const F4 d4 = __builtin_nontemporal_load(reinterpret_cast<const F4*>(p.dcur + zo * plane + cidx));
            const F4 v4 = __builtin_nontemporal_load(reinterpret_cast<const F4*>(p.v + zo * p.ldv_z + vidx));
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                dd[i] = d4[i];
                vv[i] = v4[i];
            }
        } else {
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                dd[i] = bload<kNonTemporal>(rd, coff[i]);
                vv[i] = bload<kNonTemporal>(rv, voff[i]);
            }
        }
    };
    float q[M][4];      // u(z'') of the thread's points at slot (z'' - z_begin) mod M
    float acc[Q][4];    // partial sum of output o at slot (o - z_begin) mod Q
#pragma unroll
    for (int k = 0; k < M; ++k)
#pragma unroll
        for (int i = 0; i < 4; ++i) q[k][i] = 0.f;
#pragma unroll
    for (int k = 0; k < Q; ++k)
#pragma unroll
        for (int i = 0; i < 4; ++i) acc[k][i] = 0.f;
    // the finished update of a plane: stored at once (AHEAD), else after the
    // next barrier
    float pd[4], pu[4];
    bool pending = false;
    Rsrc pst_d = plane_rsrc_at(0, 0u), pst_u = plane_rsrc_at(0, 0u);
    auto flush = [&]() {
        if (!pending) return;
        if constexpr (VEC) {
            U4 d4, u4;
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                d4[i] = __builtin_bit_cast(unsigned, pd[i]);
                u4[i] = __builtin_bit_cast(unsigned, pu[i]);
            }
            bstore4_nt(d4, pst_d, coff[0]);
            bstore4_nt(u4, pst_u, coff[0]);
        } else {
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                bstore_nt(pd[i], pst_d, coff[i]);
                bstore_nt(pu[i], pst_u, coff[i]);
            }
        }
        pending = false;
    };
    load_plane_lds(lds);
    if constexpr (AHEAD) fetch_dv(dv[0][0], dv[0][1]);   // output z_begin - M
    auto body = [&](auto ph, int zp) {
        constexpr int PH = decltype(ph)::value;
        float* cur = lds + (PH & 1) * PLANE;
        // this wave's loads into LDS (and every other memory operation it has
        // in flight) complete, then the barrier: plane zp is in cur, and every
        // thread is done with the other buffer
        if constexpr (AHEAD) {
            // the stores of the previous plane, issued last, may stay in flight
            constexpr int NS = VEC ? 2 : 8;
            __builtin_amdgcn_s_waitcnt(0x0F70 | NS);   // vmcnt(NS)
        } else {
            __builtin_amdgcn_s_waitcnt(0x0F70);   // vmcnt(0)
        }
        __syncthreads();
        float* nxt = lds + ((PH & 1) ^ 1) * PLANE;
        constexpr int DV = AHEAD ? PH & 1 : 0;   // slot of output zp - M
        if constexpr (AHEAD) {
            fetch_dv(dv[DV ^ 1][0], dv[DV ^ 1][1]);   // output zp + 1 - M
        } else {
            if (zp + 1 < z_end) load_plane_lds(nxt);
            fetch_dv(dv[0][0], dv[0][1]);   // output zp - M
        }
        if constexpr (!AHEAD) flush();
        float S[NG][4], uc[4];
        ball_rows_from<M, MP, LW, Q, PH, 0, NG>(cur + (ty + M) * LW + 4 * tq, S, uc, acc, p.w);
        if constexpr (AHEAD) {
            if (zp + 1 < z_end) load_plane_lds(nxt);
        }
        const float (&dd)[4] = dv[DV][0];
        const float (&vv)[4] = dv[DV][1];
        // z differences: output zp - m and output zp
        cfor<1, M + 1>([&](auto mc) {
            constexpr int m = decltype(mc)::value;
            constexpr int qs_ = ((PH - m) % M + M) % M, as = ((PH - m) % Q + Q) % Q;
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const float dl = uc[i] - q[qs_][i];
                acc[as][i] = fmaf(p.w.wc[m], dl, acc[as][i]);
                acc[PH][i] = fmaf(-p.w.wc[m], dl, acc[PH][i]);
            }
        });
        // output o = zp - M is complete
        constexpr int QO = PH % M, AO = (PH + M) % Q;
        const int o = zp - M;
        const bool oin = o >= zs && o < ze;
        if (AHEAD || oin) {
            const int dzb = nb > 0 ? band_depth(o, p.nz, nb) : 0;
            const float rz = dzb * p.sp.inv_nb;
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const bool inband = xyband[i] || dzb != 0;
                const float e = inband ? p.sp.escale * fmaf(rz, rz, exy[i]) : 0.f;
                const float d = delta_update(dd[i], vv[i], acc[AO][i], inband, e, src_i == i && o == src_z, qs);
                pd[i] = d;
                pu[i] = q[QO][i] + d;
            }
            pst_d = plane_rsrc_at(adn, oin ? pbytes : 0u);
            pst_u = plane_rsrc_at(aun, oin ? pbytes : 0u);
            pending = true;
        }
        if constexpr (AHEAD) flush();   // every plane, in or out of the chunk: a fixed count
        adn += pstep;
        aun += pstep;
#pragma unroll
        for (int i = 0; i < 4; ++i) q[QO][i] = uc[i];
    };
    for (int z = z_begin; z < z_end; z += Q) run_phases<0, Q>(body, z, z_end);
    flush();
}

template <int SHAPE, int M, int RY>
__global__ __launch_bounds__(kBlock3) void k_adj3d_gen(AdjArgs p) {
    using G = Geo3<M, RY>;
    constexpr int NP = 2 * M + 1;
    __shared__ RingLDS<SHAPE, M, RY, 2> L;
    float* rp = &L.f[0][0][0];
    float* ru = &L.f[1][0][0];
    const Pos3 b = block_pos<RY>(p.ntiles, p.tiles_x, p.tiles_y, p.zchunk, p.nz);
    for (int i = 0; i < 2 * M; ++i) {
        load_plane<M, RY>(rp + i * G::PLANE, p.pcur, p.nx, p.ny, p.nz, b.x0, b.y0, b.zs - M + i);
        if (p.with_grad)
            load_plane<M, RY>(ru + i * G::PLANE, p.ufwd, p.nx, p.ny, p.nz, b.x0, b.y0, b.zs - M + i);
    }
    int base = M;
    for (int z = b.zs; z < b.ze; ++z) {
        int front = base + M;
        if (front >= NP) front -= NP;
        load_plane<M, RY>(rp + front * G::PLANE, p.pcur, p.nx, p.ny, p.nz, b.x0, b.y0, z + M);
        if (p.with_grad)
            load_plane<M, RY>(ru + front * G::PLANE, p.ufwd, p.nx, p.ny, p.nz, b.x0, b.y0, z + M);
        float pp[RY], vv[RY], gg[RY];
#pragma unroll
        for (int j = 0; j < RY; ++j) {
            const int gy = b.y0 + b.ty * RY + j;
            const bool ok = b.gx < p.nx && gy < p.ny;
            const long long k = ((long long)z * p.ny + gy) * p.nx + b.gx;
            const long long kv = (long long)z * p.ldv_z + (long long)gy * p.ldv_y + b.gx;
            pp[j] = (ok && p.with_update) ? p.pprev[k] : 0.f;
            vv[j] = ok ? p.v[kv] : 0.f;
            gg[j] = (ok && p.with_grad) ? p.grad[kv] : 0.f;
        }
        __syncthreads();
#pragma unroll
        for (int j = 0; j < RY; ++j) {
            const int row = b.ty * RY + j + M, col = b.tx + M;
            const float pc = rp[base * G::PLANE + row * G::LW + col];
            float Lp = 0.f, Lu = 0.f;
            gen_layers<SHAPE, M, RY, 0>(rp, base, row, col, pc, Lp, p.w);
            if (p.with_grad) {
                const float uc = ru[base * G::PLANE + row * G::LW + col];
                gen_layers<SHAPE, M, RY, 0>(ru, base, row, col, uc, Lu, p.w);
            }
            const int gy = b.y0 + b.ty * RY + j;
            if (b.gx < p.nx && gy < p.ny) {
                const long long k = ((long long)z * p.ny + gy) * p.nx + b.gx;
                const long long kv = (long long)z * p.ldv_z + (long long)gy * p.ldv_y + b.gx;
                if (p.with_grad) p.grad[kv] = fmaf(grad_factor(p.gparam, p.gscale, vv[j]) * pc, Lu, gg[j]);
                if (p.with_update) {
                    bool inband;
                    const float e = damp_e(p.sp, b.gx, gy, z, p.nx, p.ny, p.nz, inband);
                    float r;
                    if (!inband) {
                        r = fmaf(vv[j], Lp, 2.f * pc - pp[j]);
                    } else {
                        r = fmaf(-(1.f - e), pp[j], 2.f * pc);
                        r = fmaf(vv[j], Lp, r);
                        r = r / (1.f + e);
                    }
                    p.pnext[k] = r;
                }
            }
        }
        __syncthreads();
        base = base + 1 == NP ? 0 : base + 1;
    }
}

}  // namespace

// ---------------------------------------------------------------------------
// dispatch.  Compiled forward variants: cross M = 1..8 with rows 1, 2, 4;
// rhombus and square M = 1..4 with rows 1, 2; rhombus M = 5, 6 with rows 1.
// Adjoint: cross M = 1..8 (forward rows), rhombus M = 1..4 and square
// M = 1, 2 with rows 1.
// ---------------------------------------------------------------------------
bool have_fwd3d(int shape, int M, int rows) {
    if (shape == SH_CROSS) return M >= 1 && M <= 8 && (rows == 1 || rows == 2 || rows == 4);
    if (shape == SH_RHOMBUS || shape == SH_SQUARE) {
        if (M >= 1 && M <= 4) return rows == 1 || rows == 2;
        if (shape == SH_RHOMBUS && (M == 5 || M == 6)) return rows == 1;
    }
    return false;
}

template <int M, int RY>
static void run_cross(const StepArgs& a, hipStream_t s) {
    if (planes_fit(a))
        hipLaunchKernelGGL((k_fwd3d_cross<M, RY>), dim3(a.ntiles), dim3(kBlock3), 0, s, a);
    else
        hipLaunchKernelGGL((k_fwd3d_cross_wide<M, RY>), dim3(a.ntiles), dim3(kBlock3), 0, s, a);
}
template <int M, int RY>
static void run_cross_adj(const AdjArgs& a, hipStream_t s) {
    if ((long long)a.nx * a.ny < (1LL << 29) && a.ldv_z < (1LL << 29))
        hipLaunchKernelGGL((k_adj3d_cross<M, RY>), dim3(a.ntiles), dim3(kBlock3), 0, s, a);
    else
        hipLaunchKernelGGL((k_adj3d_cross_wide<M, RY>), dim3(a.ntiles), dim3(kBlock3), 0, s, a);
}
template <int SHAPE, int M, int RY>
static void run_gen(const StepArgs& a, hipStream_t s) {
    hipLaunchKernelGGL((k_fwd3d_gen<SHAPE, M, RY>), dim3(a.ntiles), dim3(kBlock3), 0, s, a);
}
template <int SHAPE, int M, int RY>
static void run_gen_adj(const AdjArgs& a, hipStream_t s) {
    hipLaunchKernelGGL((k_adj3d_gen<SHAPE, M, RY>), dim3(a.ntiles), dim3(kBlock3), 0, s, a);
}

template <int M>
static bool cross_rows(const StepArgs& a, int rows, hipStream_t s) {
    switch (rows) {
        case 1: run_cross<M, 1>(a, s); return true;
        case 2: run_cross<M, 2>(a, s); return true;
        case 4: run_cross<M, 4>(a, s); return true;
    }
    return false;
}
template <int M>
static bool cross_rows_adj(const AdjArgs& a, int rows, hipStream_t s) {
    switch (rows) {
        case 1: run_cross_adj<M, 1>(a, s); return true;
        case 2: run_cross_adj<M, 2>(a, s); return true;
        case 4: run_cross_adj<M, 4>(a, s); return true;
    }
    return false;
}
// The ball kernel tiles 64 x 4W points (W waves; rows = 1: W = 4, rows = 2:
// W = 8) and takes its own tile grid.
template <int M, int W>
static void run_ball(const StepArgs& a, hipStream_t s) {
    StepArgs b = a;
    constexpr int TY = BallGeo<M, W>::TY;
    b.tiles_x = (a.nx + 63) / 64;
    b.tiles_y = (a.ny + TY - 1) / TY;
    b.ntiles = b.tiles_x * b.tiles_y * ((a.nz + a.zchunk - 1) / a.zchunk);
    auto al16 = [](const void* q) { return ((uintptr_t)q & 15) == 0; };
    const bool vec = a.nx % 4 == 0 && a.ldv_y % 4 == 0 && a.ldv_z % 4 == 0 && al16(a.ucur) && al16(a.dcur) &&
                     al16(a.dnext) && al16(a.unext) && al16(a.v);
    if (vec)
        hipLaunchKernelGGL((k_fwd3d_ball<M, W, 1>), dim3(b.ntiles), dim3(64 * W), 0, s, b);
    else
        hipLaunchKernelGGL((k_fwd3d_ball<M, W, 0>), dim3(b.ntiles), dim3(64 * W), 0, s, b);
}
template <int M>
static bool ball_rows(const StepArgs& a, int rows, hipStream_t s) {
    if constexpr (M <= 4) {
        switch (rows) {
            case 1: run_ball<M, 4>(a, s); return true;
            case 2: run_ball<M, 8>(a, s); return true;
        }
        return false;
    } else {
        if (rows != 1) return false;
        run_ball<M, 4>(a, s);
        return true;
    }
}

template <int SHAPE, int M>
static bool gen_rows(const StepArgs& a, int rows, hipStream_t s) {
    if constexpr (M <= 4) {
        switch (rows) {
            case 1: run_gen<SHAPE, M, 1>(a, s); return true;
            case 2: run_gen<SHAPE, M, 2>(a, s); return true;
        }
        return false;
    } else {
        if (rows != 1) return false;
        run_gen<SHAPE, M, 1>(a, s);
        return true;
    }
}

bool launch_fwd3d(const StepArgs& a, int shape, int M, int rows, hipStream_t s) {
    if (!have_fwd3d(shape, M, rows)) return false;
    if (shape == SH_CROSS) {
        switch (M) {
            case 1: return cross_rows<1>(a, rows, s);
            case 2: return cross_rows<2>(a, rows, s);
            case 3: return cross_rows<3>(a, rows, s);
            case 4: return cross_rows<4>(a, rows, s);
            case 5: return cross_rows<5>(a, rows, s);
            case 6: return cross_rows<6>(a, rows, s);
            case 7: return cross_rows<7>(a, rows, s);
            case 8: return cross_rows<8>(a, rows, s);
        }
        return false;
    }
    if (shape == SH_RHOMBUS && planes_fit(a)) {   // the L1 ball: in-plane sums reused along z
        switch (M) {
            case 1: return ball_rows<1>(a, rows, s);
            case 2: return ball_rows<2>(a, rows, s);
            case 3: return ball_rows<3>(a, rows, s);
            case 4: return ball_rows<4>(a, rows, s);
            case 5: return ball_rows<5>(a, rows, s);
            case 6: return ball_rows<6>(a, rows, s);
        }
        return false;
    }
    if (shape == SH_RHOMBUS) {
        switch (M) {
            case 1: return gen_rows<SH_RHOMBUS, 1>(a, rows, s);
            case 2: return gen_rows<SH_RHOMBUS, 2>(a, rows, s);
            case 3: return gen_rows<SH_RHOMBUS, 3>(a, rows, s);
            case 4: return gen_rows<SH_RHOMBUS, 4>(a, rows, s);
            case 5: return gen_rows<SH_RHOMBUS, 5>(a, rows, s);
            case 6: return gen_rows<SH_RHOMBUS, 6>(a, rows, s);
        }
        return false;
    }
    switch (M) {
        case 1: return gen_rows<SH_SQUARE, 1>(a, rows, s);
        case 2: return gen_rows<SH_SQUARE, 2>(a, rows, s);
        case 3: return gen_rows<SH_SQUARE, 3>(a, rows, s);
        case 4: return gen_rows<SH_SQUARE, 4>(a, rows, s);
    }
    return false;
}

// The adjoint uses the forward tile height for crosses; rhombus and square
// adjoints always run with one row per thread (two rings of planes in LDS).
bool launch_adj3d(const AdjArgs& a, int shape, int M, int rows, hipStream_t s) {
    if (shape == SH_CROSS) {
        switch (M) {
            case 1: return cross_rows_adj<1>(a, rows, s);
            case 2: return cross_rows_adj<2>(a, rows, s);
            case 3: return cross_rows_adj<3>(a, rows, s);
            case 4: return cross_rows_adj<4>(a, rows, s);
            case 5: return cross_rows_adj<5>(a, rows, s);
            case 6: return cross_rows_adj<6>(a, rows, s);
            case 7: return cross_rows_adj<7>(a, rows, s);
            case 8: return cross_rows_adj<8>(a, rows, s);
        }
        return false;
    }
    if (rows != 1) return false;
    if (shape == SH_RHOMBUS) {
        switch (M) {
            case 1: run_gen_adj<SH_RHOMBUS, 1, 1>(a, s); return true;
            case 2: run_gen_adj<SH_RHOMBUS, 2, 1>(a, s); return true;
            case 3: run_gen_adj<SH_RHOMBUS, 3, 1>(a, s); return true;
            case 4: run_gen_adj<SH_RHOMBUS, 4, 1>(a, s); return true;
        }
        return false;
    }
    switch (M) {
        case 1: run_gen_adj<SH_SQUARE, 1, 1>(a, s); return true;
        case 2: run_gen_adj<SH_SQUARE, 2, 1>(a, s); return true;
    }
    return false;
}

bool have_adj3d(int shape, int M) {
    if (shape == SH_CROSS) return M >= 1 && M <= 8;
    if (shape == SH_RHOMBUS) return M >= 1 && M <= 4;
    return shape == SH_SQUARE && M >= 1 && M <= 2;
}

// The cross adjoint reads two fields with halos per plane; for M <= 4 it runs
// faster on taller tiles than the forward (512^3 FWI gradient at M4: 313 vs
// 330 ms per 200 steps), while at larger radii taller tiles spill (M8 at 4
// rows: 2.6x slower) and it keeps the forward's choice.
int adj_rows3d(int shape, int M, int fwd_rows) {
    if (shape != SH_CROSS) return 1;
    return M <= 4 ? 4 : fwd_rows;
}

}  // namespace fdw
