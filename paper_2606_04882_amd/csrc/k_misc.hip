// Small helper kernels: coefficient preparation, fills, copies, receiver
// indexing, trace gather, adjoint source injection and a finiteness check.
// All are grid-stride loops over at most a few model-sized arrays.
#include "fd_kernels.h"

namespace fdw {

static inline int grid_for(long long n) {
    long long b = (n + kBlock - 1) / kBlock;
    if (b < 1) b = 1;
    if (b > 65536) b = 65536;
    return (int)b;
}

// v = (c dt / h)^2 formed in FP64 and rounded once to FP32 (the squared
// Courant number of Sec. 3.4.1, eq. courant); non-positive or non-finite
// velocities are counted in flags[FLAG_BAD_VEL], velocities whose Courant
// number c dt / h exceeds c_lim (the stability limit of eq. full_disp) in
// flags[FLAG_UNSTABLE_VEL].
__global__ void k_vprep(const float* __restrict__ vel, float* __restrict__ v, long long n,
                        double dt_over_h, double c_lim, int* __restrict__ flags) {
    for (long long i = blockIdx.x * (long long)kBlock + threadIdx.x; i < n;
         i += (long long)gridDim.x * kBlock) {
        const float c = vel[i];
        if (!(c > 0.f) || !isfinite(c)) atomicAdd(&flags[FLAG_BAD_VEL], 1);
        const double t = (double)c * dt_over_h;
        if (t > c_lim) atomicAdd(&flags[FLAG_UNSTABLE_VEL], 1);
        v[i] = (float)(t * t);
    }
}

__global__ void k_fill(float* __restrict__ p, long long n, float val) {
    for (long long i = blockIdx.x * (long long)kBlock + threadIdx.x; i < n;
         i += (long long)gridDim.x * kBlock)
        p[i] = val;
}

__global__ void k_fill_i32(int* __restrict__ p, long long n, int val) {
    for (long long i = blockIdx.x * (long long)kBlock + threadIdx.x; i < n;
         i += (long long)gridDim.x * kBlock)
        p[i] = val;
}

__global__ void k_copy(float* __restrict__ dst, const float* __restrict__ src, long long n) {
    for (long long i = blockIdx.x * (long long)kBlock + threadIdx.x; i < n;
         i += (long long)gridDim.x * kBlock)
        dst[i] = src[i];
}

// 16-byte accesses for fields whose pointers are 16-byte aligned
__global__ void k_copy4(float4* __restrict__ dst, const float4* __restrict__ src, long long n4) {
    for (long long i = blockIdx.x * (long long)kBlock + threadIdx.x; i < n4;
         i += (long long)gridDim.x * kBlock)
        dst[i] = src[i];
}

__global__ void k_fill4(float4* __restrict__ p, long long n4, float val) {
    for (long long i = blockIdx.x * (long long)kBlock + threadIdx.x; i < n4;
         i += (long long)gridDim.x * kBlock)
        p[i] = make_float4(val, val, val, val);
}

// window coordinates (x[, y], z) -> linear window index, or -1 (flagged)
__global__ void k_rec_index(const int* __restrict__ rec, int nrec, int ndim, int nx, int ny,
                            int nz, long long* __restrict__ lin, int* __restrict__ flags) {
    for (int r = blockIdx.x * kBlock + threadIdx.x; r < nrec; r += gridDim.x * kBlock) {
        const int x = rec[r * ndim];
        const int y = ndim == 3 ? rec[r * ndim + 1] : 0;
        const int z = rec[r * ndim + ndim - 1];
        long long idx = -1;
        if (x >= 0 && x < nx && y >= 0 && y < ny && z >= 0 && z < nz)
            idx = ((long long)z * ny + y) * nx + x;
        else
            atomicAdd(&flags[FLAG_BAD_REC], 1);
        lin[r] = idx;
    }
}

__global__ void k_gather(const float* __restrict__ u, const long long* __restrict__ lin, int nrec,
                         float* __restrict__ out) {
    for (int r = blockIdx.x * kBlock + threadIdx.x; r < nrec; r += gridDim.x * kBlock) {
        const long long i = lin[r];
        out[r] = i >= 0 ? u[i] : 0.f;
    }
}

// psi(x_r) += b(x_r) v(x_r) rho_r: the adjoint source of step k (the
// receiver residuals of trace k-1), added after the adjoint step kernel.
__global__ void k_inject(float* __restrict__ psi, const long long* __restrict__ lin, int nrec,
                         const float* __restrict__ rho, const float* __restrict__ v,
                         long long ldv_y, long long ldv_z, Sponge sp, int nx, int ny, int nz) {
    for (int r = blockIdx.x * kBlock + threadIdx.x; r < nrec; r += gridDim.x * kBlock) {
        const long long i = lin[r];
        if (i < 0) continue;
        const int x = (int)(i % nx);
        const long long t = i / nx;
        const int y = (int)(t % ny);
        const int z = (int)(t / ny);
        const float vv = v[(long long)z * ldv_z + (long long)y * ldv_y + x];
        float e = 0.f;
        if (sp.nb > 0) {
            const float rx = band_depth(x, nx, sp.nb) * sp.inv_nb;
            const float rz = band_depth(z, nz, sp.nb) * sp.inv_nb;
            float s = fmaf(rx, rx, rz * rz);
            if (ny > 1) {
                const float ry = band_depth(y, ny, sp.nb) * sp.inv_nb;
                s = fmaf(ry, ry, s);
            }
            e = sp.escale * s;
        }
        atomicAdd(&psi[i], vv * rho[r] / (1.f + e));
    }
}

__global__ void k_check_finite(const float* __restrict__ p, long long n, int* __restrict__ flags) {
    int bad = 0;
    for (long long i = blockIdx.x * (long long)kBlock + threadIdx.x; i < n;
         i += (long long)gridDim.x * kBlock)
        bad += !isfinite(p[i]);
    if (bad) atomicAdd(&flags[FLAG_NONFINITE], bad);
}

__global__ void k_accum2d(float* __restrict__ g, long long ldg, const float* __restrict__ a, int nx,
                          long long n) {
    for (long long i = blockIdx.x * (long long)kBlock + threadIdx.x; i < n;
         i += (long long)gridDim.x * kBlock) {
        const long long z = i / nx, x = i - z * nx;
        g[z * ldg + x] += a[i];
    }
}

void launch_accum2d(float* g, long long ldg, const float* a, int nx, int nz, hipStream_t s) {
    const long long n = (long long)nx * nz;
    if (n > 0) hipLaunchKernelGGL(k_accum2d, dim3(grid_for(n)), dim3(kBlock), 0, s, g, ldg, a, nx, n);
}

void launch_vprep(const float* vel, float* v, long long n, double dt_over_h, double c_lim, int* flags,
                  hipStream_t s) {
    hipLaunchKernelGGL(k_vprep, dim3(grid_for(n)), dim3(kBlock), 0, s, vel, v, n, dt_over_h, c_lim, flags);
}
void launch_fill(float* p, long long n, float val, hipStream_t s) {
    if (n <= 0) return;
    long long head = 0;
    if (((uintptr_t)p & 15) == 0 && n >= 4) {
        head = n & ~3LL;
        hipLaunchKernelGGL(k_fill4, dim3(grid_for(head / 4)), dim3(kBlock), 0, s, (float4*)p, head / 4, val);
    }
    if (head < n) hipLaunchKernelGGL(k_fill, dim3(grid_for(n - head)), dim3(kBlock), 0, s, p + head, n - head, val);
}
void launch_fill_i32(int* p, long long n, int val, hipStream_t s) {
    if (n > 0) hipLaunchKernelGGL(k_fill_i32, dim3(grid_for(n)), dim3(kBlock), 0, s, p, n, val);
}
void launch_copy(float* dst, const float* src, long long n, hipStream_t s) {
    if (n <= 0) return;
    long long head = 0;
    if ((((uintptr_t)dst | (uintptr_t)src) & 15) == 0 && n >= 4) {
        head = n & ~3LL;
        hipLaunchKernelGGL(k_copy4, dim3(grid_for(head / 4)), dim3(kBlock), 0, s, (float4*)dst,
                           (const float4*)src, head / 4);
    }
    if (head < n)
        hipLaunchKernelGGL(k_copy, dim3(grid_for(n - head)), dim3(kBlock), 0, s, dst + head, src + head, n - head);
}
void launch_rec_index(const int* rec, int nrec, int ndim, int nx, int ny, int nz,
                      long long* lin, int* flags, hipStream_t s) {
    if (nrec > 0)
        hipLaunchKernelGGL(k_rec_index, dim3(grid_for(nrec)), dim3(kBlock), 0, s, rec, nrec, ndim,
                           nx, ny, nz, lin, flags);
}
void launch_gather(const float* u, const long long* lin, int nrec, float* out, hipStream_t s) {
    if (nrec > 0)
        hipLaunchKernelGGL(k_gather, dim3(grid_for(nrec)), dim3(kBlock), 0, s, u, lin, nrec, out);
}
void launch_inject(float* psi, const long long* lin, int nrec, const float* rho, const float* v,
                   long long ldv_y, long long ldv_z, Sponge sp, int nx, int ny, int nz,
                   hipStream_t s) {
    if (nrec > 0)
        hipLaunchKernelGGL(k_inject, dim3(grid_for(nrec)), dim3(kBlock), 0, s, psi, lin, nrec, rho,
                           v, ldv_y, ldv_z, sp, nx, ny, nz);
}
void launch_check_finite(const float* p, long long n, int* flags, hipStream_t s) {
    if (n > 0)
        hipLaunchKernelGGL(k_check_finite, dim3(grid_for(n) > 1024 ? 1024 : grid_for(n)),
                           dim3(kBlock), 0, s, p, n, flags);
}

}  // namespace fdw
