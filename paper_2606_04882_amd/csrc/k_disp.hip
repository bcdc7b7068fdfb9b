// Dispersion metrics of seismic traces (Appendix A): the DFT measure gamma^F
// and the Morlet CWT measure gamma^W between numerical and reference traces.
//
// Host flow per chunk of receivers: traces [nt][nrec] are transposed into
// FP64 rows; rocFFT gives the half spectra A_k (k = 0..nt/2) of both traces;
// k_gamma_dft forms gamma^F_k = wrap(phi_num - phi_ref)/pi |A_num|/max|A_num|
// and the per-trace norm sqrt(1/nt sum_k gamma_k^2), the bins above nt/2
// being the conjugates of those below (same amplitude, opposite phase
// difference).  For the CWT, k_cwt_spectra multiplies A_k by the Morlet
// spectrum Psi*(s_j w_k) = (2 pi s_j/dt)^(1/2) pi^(-1/4) exp(-(s_j w_k - w0)^2/2)
// on the positive frequencies (H removes the rest), rocFFT's unnormalised
// inverse transform gives W_n(s_j), and k_gamma_cwt reduces
// gamma^W = wrap(phi_num - phi_ref)/pi |W_num|/max|W_num| to its norm.
// Amplitudes are sqrt(Re^2 + Im^2), phases atan2(Im, Re).  Trace rows are
// read with a row stride, so a finer run's traces can be sampled in place.
// Also here: the error norms of a numerical field or trace against a
// reference read through strides (Sec. 6.1.1).
#include "fd_kernels.h"

namespace fdw {

namespace {

constexpr int kT = 32;   // transpose tile

// out[r - r0][n] = (double) in[n * ld + r] for r in [r0, r0 + rc)
__global__ void k_rows_f64(const float* __restrict__ in, double* __restrict__ out, int nt, long long ld,
                           int r0, int rc) {
    __shared__ float t[kT][kT + 1];
    const int n0 = blockIdx.x * kT, rr0 = blockIdx.y * kT;
    const int tx = threadIdx.x, ty = threadIdx.y;   // 32 x 8 threads
    for (int i = ty; i < kT; i += 8) {
        const int n = n0 + i, r = rr0 + tx;
        t[i][tx] = (n < nt && r < rc) ? in[(long long)n * ld + r0 + r] : 0.f;
    }
    __syncthreads();
    for (int i = ty; i < kT; i += 8) {
        const int r = rr0 + i, n = n0 + tx;
        if (r < rc && n < nt) out[(long long)r * nt + n] = (double)t[tx][i];
    }
}

__device__ __forceinline__ double wrap_pi(double d) {
    if (d > M_PI) d -= 2.0 * M_PI;
    if (d < -M_PI) d += 2.0 * M_PI;
    return d;
}

__device__ __forceinline__ double amp(double2 z) { return sqrt(z.x * z.x + z.y * z.y); }

// block-wide max / sum over 256 threads
__device__ __forceinline__ double block_max(double v, double* sh) {
    sh[threadIdx.x] = v;
    __syncthreads();
    for (int s = blockDim.x / 2; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) sh[threadIdx.x] = fmax(sh[threadIdx.x], sh[threadIdx.x + s]);
        __syncthreads();
    }
    const double r = sh[0];
    __syncthreads();
    return r;
}

__device__ __forceinline__ double block_sum(double v, double* sh) {
    sh[threadIdx.x] = v;
    __syncthreads();
    for (int s = blockDim.x / 2; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) sh[threadIdx.x] += sh[threadIdx.x + s];
        __syncthreads();
    }
    const double r = sh[0];
    __syncthreads();
    return r;
}

// one block per receiver of the chunk; A, B: [rc][nh] half spectra
__global__ __launch_bounds__(256) void k_gamma_dft(const double2* __restrict__ A, const double2* __restrict__ B,
                                                    int nt, int nh, float* __restrict__ gamma, long long ldg,
                                                    double* __restrict__ norm) {
    __shared__ double sh[256];
    const int r = blockIdx.x;
    const double2* a = A + (long long)r * nh;
    const double2* b = B + (long long)r * nh;
    double m = 0.0;
    for (int k = threadIdx.x; k < nh; k += blockDim.x) m = fmax(m, amp(a[k]));
    m = block_max(m, sh);
    double s2 = 0.0;
    for (int k = threadIdx.x; k < nh; k += blockDim.x) {
        const double2 x = a[k], y = b[k];
        const double d = wrap_pi(atan2(x.y, x.x) - atan2(y.y, y.x));
        const double g = m > 0.0 ? d / M_PI * amp(x) / m : 0.0;
        const bool mirrored = k > 0 && 2 * k != nt;   // bin nt - k holds the conjugates
        s2 += (mirrored ? 2.0 : 1.0) * g * g;
        if (gamma) {
            gamma[r * ldg + k] = (float)g;
            if (mirrored) gamma[r * ldg + (nt - k)] = (float)(-g);
        }
    }
    s2 = block_sum(s2, sh);
    if (threadIdx.x == 0) norm[r] = sqrt(s2 / nt);
}

// W[(r * ns + j) * nt + k] = A[r * nh + k] Psi*(s_j w_k) for 1 <= k <= nt/2, 0 otherwise
__global__ void k_cwt_spectra(const double2* __restrict__ A, int nt, int nh, int ns, double dt, double omega0,
                              double2* __restrict__ W) {
    const int r = blockIdx.z, j = blockIdx.y;
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= nt) return;
    const double c = omega0 + sqrt(2.0 + omega0 * omega0);
    const double f = (double)(j + 1) / (nt * dt);
    const double s = c / (4.0 * M_PI * f);
    double2 out = make_double2(0.0, 0.0);
    if (k >= 1 && 2 * k <= nt) {
        const double w = 2.0 * M_PI * k / (nt * dt);
        const double e = s * w - omega0;
        const double psi = sqrt(2.0 * M_PI * s / dt) * 0.75112554446494248 * exp(-0.5 * e * e);   // pi^(-1/4)
        const double2 a = A[(long long)r * nh + k];
        out = make_double2(a.x * psi, a.y * psi);
    }
    W[((long long)r * ns + j) * nt + k] = out;
}

// one block per receiver: Wn, Wr [rc][ns][nt]
__global__ __launch_bounds__(256) void k_gamma_cwt(const double2* __restrict__ Wn, const double2* __restrict__ Wr,
                                                    long long per, double* __restrict__ norm) {
    __shared__ double sh[256];
    const int r = blockIdx.x;
    const double2* a = Wn + (long long)r * per;
    const double2* b = Wr + (long long)r * per;
    double m = 0.0;
    for (long long i = threadIdx.x; i < per; i += blockDim.x) m = fmax(m, amp(a[i]));
    m = block_max(m, sh);
    double s2 = 0.0;
    for (long long i = threadIdx.x; i < per; i += blockDim.x) {
        const double2 x = a[i], y = b[i];
        const double d = wrap_pi(atan2(x.y, x.x) - atan2(y.y, y.x));
        const double g = m > 0.0 ? d / M_PI * amp(x) / m : 0.0;
        s2 += g * g;
    }
    s2 = block_sum(s2, sh);
    if (threadIdx.x == 0) norm[r] = sqrt(s2 / (double)per);
}

// Error norms (Sec. 6.1.1) between two strided views of one box: element
// (i, j, k) of num at i sn[0] + j sn[1] + k sn[2], of ref likewise with sr.
// Each block writes (sum |e|, sum e^2, max |e|) to partial[3 b .. 3 b + 2];
// one block then reduces the partials in a fixed order (deterministic).
struct Box3 {
    long long n[3], sn[3], sr[3];
};

__global__ __launch_bounds__(256) void k_error_partials(const float* __restrict__ num, const float* __restrict__ ref,
                                                        Box3 b, double* __restrict__ partial) {
    __shared__ double sh[256];
    const long long total = b.n[0] * b.n[1] * b.n[2];
    double s1 = 0.0, s2 = 0.0, mx = 0.0;
    for (long long t = blockIdx.x * 256LL + threadIdx.x; t < total; t += (long long)gridDim.x * 256) {
        const long long i = t % b.n[0], jk = t / b.n[0];
        const long long j = jk % b.n[1], k = jk / b.n[1];
        const double e = (double)num[i * b.sn[0] + j * b.sn[1] + k * b.sn[2]] -
                         (double)ref[i * b.sr[0] + j * b.sr[1] + k * b.sr[2]];
        s1 += fabs(e);
        s2 += e * e;
        mx = fmax(mx, fabs(e));
    }
    s1 = block_sum(s1, sh);
    s2 = block_sum(s2, sh);
    mx = block_max(mx, sh);
    if (threadIdx.x == 0) {
        partial[3 * blockIdx.x] = s1;
        partial[3 * blockIdx.x + 1] = s2;
        partial[3 * blockIdx.x + 2] = mx;
    }
}

__global__ __launch_bounds__(256) void k_error_final(const double* __restrict__ partial, int nblocks,
                                                     double* __restrict__ out) {
    __shared__ double sh[256];
    double s1 = 0.0, s2 = 0.0, mx = 0.0;
    for (int b = threadIdx.x; b < nblocks; b += 256) {
        s1 += partial[3 * b];
        s2 += partial[3 * b + 1];
        mx = fmax(mx, partial[3 * b + 2]);
    }
    s1 = block_sum(s1, sh);
    s2 = block_sum(s2, sh);
    mx = block_max(mx, sh);
    if (threadIdx.x == 0) {
        out[0] = s1;
        out[1] = s2;
        out[2] = mx;
    }
}

}  // namespace

void launch_rows_f64(const float* in, long long ld, double* out, int nt, int r0, int rc, hipStream_t s) {
    dim3 grid((nt + kT - 1) / kT, (rc + kT - 1) / kT);
    hipLaunchKernelGGL(k_rows_f64, grid, dim3(kT, 8), 0, s, in, out, nt, ld, r0, rc);
}

void launch_error_norms(const float* num, const long long* sn, const float* ref, const long long* sr,
                        const long long* n, double* partial, int nblocks, double* out, hipStream_t s) {
    const Box3 b{{n[0], n[1], n[2]}, {sn[0], sn[1], sn[2]}, {sr[0], sr[1], sr[2]}};
    hipLaunchKernelGGL(k_error_partials, dim3(nblocks), dim3(256), 0, s, num, ref, b, partial);
    hipLaunchKernelGGL(k_error_final, dim3(1), dim3(256), 0, s, partial, nblocks, out);
}

void launch_gamma_dft(const void* A, const void* B, int nt, int rc, float* gamma, long long ldg, double* norm,
                      hipStream_t s) {
    hipLaunchKernelGGL(k_gamma_dft, dim3(rc), dim3(256), 0, s, (const double2*)A, (const double2*)B, nt,
                       nt / 2 + 1, gamma, ldg, norm);
}

void launch_cwt_spectra(const void* A, int nt, int rc, int ns, double dt, double omega0, void* W, hipStream_t s) {
    dim3 grid((nt + 255) / 256, ns, rc);
    hipLaunchKernelGGL(k_cwt_spectra, grid, dim3(256), 0, s, (const double2*)A, nt, nt / 2 + 1, ns, dt, omega0,
                       (double2*)W);
}

void launch_gamma_cwt(const void* Wn, const void* Wr, int nt, int rc, int ns, double* norm, hipStream_t s) {
    hipLaunchKernelGGL(k_gamma_cwt, dim3(rc), dim3(256), 0, s, (const double2*)Wn, (const double2*)Wr,
                       (long long)ns * nt, norm);
}

}  // namespace fdw
