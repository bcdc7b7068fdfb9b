// 3D forward and adjoint steps.
//
// Same update as the 2D kernels (Sec. 3.1-3.2, the 3D extension noted at the
// end of Sec. 3.1), on [nz][ny][nx] windows.  A block of kWaves3 waves owns a
// 64 (x) by kWaves3*RY (y) column of the grid and marches along z through
// `zchunk` planes:
//
//  * cross stencils keep the 2M+1 values of u along z for each of the thread's
//    RY points in registers (a queue shifted once per plane) and stage only the
//    current xy plane, with an M-cell halo, in LDS for the x/y neighbours;
//  * rhombus (L1 ball) and square (cube) stencils keep a ring of 2M+1 xy planes
//    with halo in LDS.
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

// Adjoint step and gradient term (cross), pipelined like k_fwd3d_cross: the
// operands of plane z+1 (queue fronts of psi^{k+1} and u^k, psi^{k+2}, v,
// the gradient and both halos) are fetched while plane z is computed; both
// xy planes alternate between two LDS buffers (one barrier per plane).
// psi^{k+2}, v and the gradient are touched once per step and streamed
// non-temporally; psi^{k+1} and u^k stay cacheable for the neighbouring
// blocks' halo reads.  psi^k may overwrite psi^{k+2} in place: every point is
// read (fetch of its plane) before the same thread writes it.
template <int M, int RY>
__global__ __launch_bounds__(kBlock3) void k_adj3d_cross(AdjArgs p) {
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
// L1 ball (3D rhombus): in-plane difference sums reused along z
// ---------------------------------------------------------------------------
// Split each offset d = (p, dz) into its in-plane part p and dz.  The in-plane
// parts form groups (a, b), a >= b >= 0, 1 <= a + b <= M: the points
// (+-a, +-b), (+-b, +-a), n_ab of them (4 when b = 0 or a = b, else 8).  With
//     D_ab(z') = sum_{p in (a, b)} u(x + p, z') - n_ab u(x, z')
// (a small difference, formed once per plane from the LDS copy of plane z'),
// the centre-free difference form of the stencil at plane z is
//     sum_ab [ w(a,b,0) D_ab(z) + sum_{dz=1}^{M-a-b} w(a,b,dz) (D_ab(z+dz) + D_ab(z-dz)) ]
//   + sum_{dz=1}^{M} wc(dz) (u(z+dz) + u(z-dz) - 2 u(z)),
// wc(dz) = w(0,0,dz) + sum_{a+b <= M-dz} n_ab w(a,b,dz) (formed on the host in
// FP64, rounded once): the same sum as the plain form, every term a small
// difference.  Each D_ab and u value is kept in a register queue for the
// 2 (M - a - b) + 1 (resp. 2M + 1) planes that use it, so a point costs 40
// LDS reads at M = 4 instead of 129.  The z loop is unrolled by the queue
// period P = 2M + 1, so that queue entry and LDS slot of plane z' are the
// compile-time constants (z' - z0) mod P and the queues rotate by renaming
// (no register moves).  D_ab(z') is formed at iteration z' - (M - a - b), from
// plane z + M - a - b, so iteration z reads the LDS planes z .. z + M - 1;
// plane z + M - 1 is stored at the top of iteration z (interior from the u
// queue, halo fetched during iteration z - 1), into one of P >= M + 1 slots,
// so one barrier per iteration suffices.  Each z chunk first runs 2 (M - 1)
// warm-up iterations that only fill the queues.
__host__ __device__ constexpr int ball_ngroups(int M) {
    int n = 0;
    for (int s = 1; s <= M; ++s) n += s / 2 + 1;
    return n;
}
__host__ __device__ constexpr int ball_ga(int M, int g) {
    for (int s = 1; s <= M; ++s)
        for (int b = 0; b <= s / 2; ++b) {
            if (g == 0) return s - b;
            --g;
        }
    return -1;
}
__host__ __device__ constexpr int ball_gb(int M, int g) {
    for (int s = 1; s <= M; ++s)
        for (int b = 0; b <= s / 2; ++b) {
            if (g == 0) return b;
            --g;
        }
    return -1;
}
// orbit of the offset with absolute components (x, y, z), any order
__host__ __device__ constexpr int ball_orbit(int M, int x, int y, int z) {
    return orbit3_of(SH_RHOMBUS, M, x, y, z);
}

// sum of u over the in-plane group (A, B) around (row, col) of an LDS plane
template <int M, int RY, int A, int B>
__device__ __forceinline__ float ring_sum(const float* t, int row, int col) {
    constexpr int LW = Geo3<M, RY>::LW;
    const float* c = t + row * LW + col;
    if constexpr (B == 0) return (c[-A] + c[A]) + (c[-A * LW] + c[A * LW]);
    else if constexpr (A == B) return (c[-A * LW - A] + c[-A * LW + A]) + (c[A * LW - A] + c[A * LW + A]);
    else
        return ((c[-B * LW - A] + c[-B * LW + A]) + (c[B * LW - A] + c[B * LW + A])) +
               ((c[-A * LW - B] + c[-A * LW + B]) + (c[A * LW - B] + c[A * LW + B]));
}

template <int G, int NG, int M, int RY, int PH, int P>
__device__ __forceinline__ void ball_form_d(float (&D)[NG][P], const float* lds, const float (&q)[P], int row,
                                            int col) {
    if constexpr (G < NG) {
        constexpr int a = ball_ga(M, G), b = ball_gb(M, G), s = a + b, mz = M - s;
        constexpr float n = (b == 0 || a == b) ? 4.f : 8.f;
        constexpr int slot = (PH + M - s) % P;   // plane z + M - s
        const float r = ring_sum<M, RY, a, b>(lds + slot * Geo3<M, RY>::PLANE, row, col);
        D[G][(PH + mz) % P] = fmaf(-n, q[slot], r);
        ball_form_d<G + 1, NG, M, RY, PH, P>(D, lds, q, row, col);
    }
}

// w(A,B,DZ) (D(z+DZ) + D(z-DZ)) for DZ = DZ..MZ of one group's queue
template <int M, int PH, int P, int A, int B, int DZ, int MZ>
__device__ __forceinline__ float ball_dz(const float (&Dg)[P], const Weights& W, float acc) {
    if constexpr (DZ <= MZ) {
        constexpr int o = ball_orbit(M, A, B, DZ);
        acc = fmaf(W.w[o], Dg[(PH + DZ) % P] + Dg[(PH + P - DZ) % P], acc);
        return ball_dz<M, PH, P, A, B, DZ + 1, MZ>(Dg, W, acc);
    } else {
        return acc;
    }
}

template <int G, int NG, int M, int PH, int P>
__device__ __forceinline__ float ball_combine(const float (&D)[NG][P], const Weights& W, float acc) {
    if constexpr (G < NG) {
        constexpr int a = ball_ga(M, G), b = ball_gb(M, G), mz = M - a - b;
        constexpr int o = ball_orbit(M, a, b, 0);
        acc = fmaf(W.w[o], D[G][PH], acc);
        acc = ball_dz<M, PH, P, a, b, 1, mz>(D[G], W, acc);
        return ball_combine<G + 1, NG, M, PH, P>(D, W, acc);
    } else {
        return acc;
    }
}

// Window and model planes are addressed with 32-bit byte offsets below 2^31.
bool planes_fit(const StepArgs& a) {
    return (long long)a.nx * a.ny < (1LL << 29) && a.ldv_z < (1LL << 29);
}

template <int M, int RY>
__global__ __launch_bounds__(kBlock3) __attribute__((amdgpu_waves_per_eu(M <= 4 ? 4 : 2))) void k_fwd3d_ball(StepArgs p) {
    using G = Geo3<M, RY>;
    constexpr int P = 2 * M + 1;
    constexpr int NG = ball_ngroups(M);
    constexpr int WARM = 2 * (M - 1);
    __shared__ float lds[P * G::PLANE];
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
    const int z0 = b.zs - WARM;
    // the thread's columns: byte offsets in a window plane and a model plane
    float q[RY][P];        // u(z') at (z' - z0) mod P
    float D[RY][NG][P];    // D_g(z') at (z' - z0) mod P
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
#pragma unroll
        for (int k = 0; k < P; ++k) {
            q[j][k] = 0.f;
#pragma unroll
            for (int g = 0; g < NG; ++g) D[j][g][k] = 0.f;
        }
    }
    // plane z of a window field (every access of a plane off the grid reads 0)
    auto wplane = [&](const float* f, int z) {
        const bool in = (unsigned)z < (unsigned)p.nz;
        return plane_rsrc(f + (in ? z : 0) * plane, in ? pbytes : 0u);
    };
    // u(z0 - M .. z0 + M - 1) at (k mod P)
#pragma unroll
    for (int k = -M; k < M; ++k) {
        const Rsrc r = wplane(p.ucur, z0 + k);
#pragma unroll
        for (int j = 0; j < RY; ++j) q[j][(k + P) % P] = bload(r, coff[j]);
    }
    // LDS planes z0 .. z0 + M - 2 (slots 0 .. M - 2)
    for (int k = 0; k + 1 < M; ++k) load_plane<M, RY>(lds + k * G::PLANE, p.ucur, p.nx, p.ny, p.nz, b.x0, b.y0, z0 + k);
    PlaneHalo<M, RY> halo;
    halo.init(p.nx, p.ny, b.x0, b.y0);
    float front[RY], dd[RY], vv[RY];
    // byte addresses of the planes the next fetch and the next update touch:
    // u(z + M), d(z), v(z) and d/u^{n+1}(z), advanced by one plane per call
    const unsigned long long pstep = 4ull * (unsigned long long)plane, vstep = 4ull * (unsigned long long)p.ldv_z;
    unsigned long long au = (unsigned long long)p.ucur + (unsigned long long)(long long)(z0 + M) * pstep;
    unsigned long long ad = (unsigned long long)p.dcur + (unsigned long long)(long long)z0 * pstep;
    unsigned long long av = (unsigned long long)p.v + (unsigned long long)(long long)z0 * vstep;
    unsigned long long adn = (unsigned long long)p.dnext + (unsigned long long)(long long)z0 * pstep;
    unsigned long long aun = (unsigned long long)p.unext + (unsigned long long)(long long)z0 * pstep;
    auto fetch = [&](int z) {   // operands of iteration z (d and v only for the chunk's own planes)
        const bool in = z >= b.zs && z < b.ze;
        const Rsrc ru = plane_rsrc_at(au, (unsigned)(z + M) < (unsigned)p.nz ? pbytes : 0u);
        const Rsrc rh = plane_rsrc_at(au - pstep, (unsigned)(z + M - 1) < (unsigned)p.nz ? pbytes : 0u);
        const Rsrc rd = plane_rsrc_at(ad, in ? pbytes : 0u);
        const Rsrc rv = plane_rsrc_at(av, in ? vbytes : 0u);
        au += pstep;
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
    auto body = [&](auto ph, int z) {
        constexpr int PH = decltype(ph)::value;
        constexpr int S_NEW = (PH + M - 1) % P;   // slot of plane z + M - 1
        float ddc[RY], vvc[RY];
#pragma unroll
        for (int j = 0; j < RY; ++j) {
            q[j][(PH + M) % P] = front[j];
            ddc[j] = dd[j];
            vvc[j] = vv[j];
            lds[S_NEW * G::PLANE + (b.ty * RY + j + M) * G::LW + b.tx + M] = q[j][S_NEW];
        }
        halo.store(lds + S_NEW * G::PLANE);
        if (z + 1 < b.ze) fetch(z + 1);
        __syncthreads();
#pragma unroll
        for (int j = 0; j < RY; ++j)
            ball_form_d<0, NG, M, RY, PH, P>(D[j], lds, q[j], b.ty * RY + j + M, b.tx + M);
        const Rsrc rdn = plane_rsrc_at(adn, pbytes);
        const Rsrc run = plane_rsrc_at(aun, pbytes);
        adn += pstep;
        aun += pstep;
        if (z >= b.zs) {
            const int dzb = nb > 0 ? band_depth(z, p.nz, nb) : 0;
            const float rz = dzb * p.sp.inv_nb;
#pragma unroll
            for (int j = 0; j < RY; ++j) {
                const float uc = q[j][PH];
                float L = ball_combine<0, NG, M, PH, P>(D[j], p.w, 0.f);
#pragma unroll
                for (int dz = 1; dz <= M; ++dz)
                    L = fmaf(p.w.wc[dz], fmaf(-2.f, uc, q[j][(PH + dz) % P] + q[j][(PH + P - dz) % P]), L);
                const bool inband = (dxb | dyb[j] | dzb) != 0;
                const float e = inband ? p.sp.escale * fmaf(rx, rx, fmaf(ry[j], ry[j], rz * rz)) : 0.f;
                const float d = delta_update(ddc[j], vvc[j], L, inband, e, srccol[j] && z == src_z, qs);
                bstore_nt(d, rdn, coff[j]);         // lanes off the grid: dropped
                bstore_nt(uc + d, run, coff[j]);
            }
        }
    };
    for (int z = z0; z < b.ze; z += P) run_phases<0, P>(body, z, b.ze);
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
    hipLaunchKernelGGL((k_adj3d_cross<M, RY>), dim3(a.ntiles), dim3(kBlock3), 0, s, a);
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
template <int M, int RY>
static void run_ball(const StepArgs& a, hipStream_t s) {
    hipLaunchKernelGGL((k_fwd3d_ball<M, RY>), dim3(a.ntiles), dim3(kBlock3), 0, s, a);
}
template <int M>
static bool ball_rows(const StepArgs& a, int rows, hipStream_t s) {
    if constexpr (M <= 4) {
        switch (rows) {
            case 1: run_ball<M, 1>(a, s); return true;
            case 2: run_ball<M, 2>(a, s); return true;
        }
        return false;
    } else {
        if (rows != 1) return false;
        run_ball<M, 1>(a, s);
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
