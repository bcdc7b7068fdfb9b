// Internal declarations shared by the HIP kernels and the host library.
// Not part of the public ABI (see include/fdwave.h).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace fdw {

// Kernel families: cross, rhombus and square with their extents known at
// compile time, and SH_NSHAPE for the 2D cross-rhombus / cross-square
// shapes, whose dense kernels read each column's z extent from Weights::mz.
enum { SH_CROSS = 0, SH_RHOMBUS = 1, SH_SQUARE = 2, SH_NSHAPE = 3 };
constexpr int kMaxOrbits = 64;
constexpr int kBlock = 256;   // threads per block: 4 waves of 64
constexpr int kTileX = 64;    // tile width along x = one wave
// 3D kernels: waves per block; a block's tile is 64 x kWaves3 * rows in xy
constexpr int kWaves3 = 8;
constexpr int kBlock3 = 64 * kWaves3;

// FP32 weights, one per orbit in canonical order (orbit 0, the centre, is
// never read: the kernels use the centre-free difference form).  wd is the
// same weights laid out densely by 2D offset group: wd[dx*(M+1) + dz] is the
// weight of (dx, dz) (0 outside the shape), used by the dense 2D kernels.
// wc[dz] (dz = 1..M) is the weight the dense 2D kernels give the centre
// column's z difference u(z+dz) + u(z-dz) - 2u: w(0, dz) + 2 sum_dx w(dx, dz),
// formed in FP64 from the FP32 weights and rounded once.  mz[dx] (dx = 1..M)
// is the z extent of the dense 2D kernels' offset group at column dx: the
// shape holds (dx, dz) exactly for dz = 0..mz[dx] (read by SH_NSHAPE
// kernels only; the others know it at compile time).  For the cross kernels,
// w[m] is the weight of the axis offset m.
constexpr int kMaxDense = 81;
struct Weights {
    float w[kMaxOrbits];
    float wd[kMaxDense];
    float wc[9];
    int mz[9];
};

// ---------------------------------------------------------------------------
// Compile-time stencil geometry.  A 2D orbit representative is (p, q) with
// p >= q >= 0; a 3D one (p, q, r) with p >= q >= r >= 0.  Orbits are ordered
// lexicographically ascending by representative.
// ---------------------------------------------------------------------------
__host__ __device__ constexpr bool in_shape2(int shape, int M, int p, int q) {
    return shape == SH_CROSS ? (q == 0 && p <= M)
         : shape == SH_RHOMBUS ? (p + q <= M) : (p <= M);
}

__host__ __device__ constexpr int orbit2(int shape, int M, int a, int b) {
    int idx = 0;
    for (int p = 0; p <= M; ++p)
        for (int q = 0; q <= p; ++q) {
            if (p == a && q == b) return idx;
            if (in_shape2(shape, M, p, q)) ++idx;
        }
    return -1;
}

// index of the orbit containing offset (dx, dz), any signs/order
__host__ __device__ constexpr int orbit2_of(int shape, int M, int dx, int dz) {
    int a = dx < 0 ? -dx : dx, b = dz < 0 ? -dz : dz;
    return a >= b ? orbit2(shape, M, a, b) : orbit2(shape, M, b, a);
}

// largest |dz| in the shape for a given |dx|
__host__ __device__ constexpr int maxdz2(int shape, int M, int dx) {
    return shape == SH_CROSS ? (dx == 0 ? M : 0) : shape == SH_RHOMBUS ? M - dx : M;
}

__host__ __device__ constexpr bool in_shape3(int shape, int M, int p, int q, int r) {
    return shape == SH_CROSS ? (q == 0 && r == 0 && p <= M)
         : shape == SH_RHOMBUS ? (p + q + r <= M) : (p <= M);
}

__host__ __device__ constexpr int orbit3(int shape, int M, int a, int b, int c) {
    int idx = 0;
    for (int p = 0; p <= M; ++p)
        for (int q = 0; q <= p; ++q)
            for (int r = 0; r <= q; ++r) {
                if (p == a && q == b && r == c) return idx;
                if (in_shape3(shape, M, p, q, r)) ++idx;
            }
    return -1;
}

__host__ __device__ constexpr int cabs_(int x) { return x < 0 ? -x : x; }
__host__ __device__ constexpr int cmax_(int a, int b) { return a > b ? a : b; }
__host__ __device__ constexpr int cmin_(int a, int b) { return a < b ? a : b; }

__host__ __device__ constexpr int orbit3_of(int shape, int M, int dx, int dy, int dz) {
    int a = cabs_(dx), b = cabs_(dy), c = cabs_(dz);
    int hi = cmax_(a, cmax_(b, c)), lo = cmin_(a, cmin_(b, c));
    int mid = a + b + c - hi - lo;
    return orbit3(shape, M, hi, mid, lo);
}

// ---------------------------------------------------------------------------
// Block -> tile mapping.  Workgroups are dealt round-robin to the 8 XCDs;
// remap so that each XCD owns a contiguous run of tiles (neighbouring tiles
// share halo rows in that XCD's L2).
// ---------------------------------------------------------------------------
__device__ __forceinline__ int xcd_tile(int bid, int ntiles) {
    const int q = ntiles >> 3, r = ntiles & 7;
    const int xcd = bid & 7, slot = bid >> 3;
    return xcd * q + (xcd < r ? xcd : r) + slot;
}

// Damping factors for a node at band depths (dx, dy, dz) (cells):
// e = eta_max dt/2 * sum (d/nb)^2, a = 1 - e, b = 1 / (1 + e).
struct Sponge {
    int nb;
    float escale;   // eta_max * dt / 2
    float inv_nb;   // 1 / nb
};

__device__ __forceinline__ int band_depth(int i, int n, int nb) {
    int d = nb - i;
    int d2 = i - (n - 1 - nb);
    d = d > d2 ? d : d2;
    return d > 0 ? d : 0;
}

// ---------------------------------------------------------------------------
// Time stepping in difference form.  The forward state at step n is the pair
// (u^n, d^n), d^n = u^n - u^{n-1}: with a = 1 - e, b = 1 / (1 + e) the
// leapfrog update b [2 u^n - a u^{n-1} + v L + q s] (Sec. 3.2 eq.
// time_derivative1 with the damping term of Sec. 3.1) is, exactly,
//     d^{n+1} = [(1 - e) d^n + v L + q s] / (1 + e),   u^{n+1} = u^n + d^{n+1}.
// Storing d instead of u^{n-1} keeps the per-step change at full FP32
// precision: with many time steps per period the change is a small fraction
// of u, and u^{n+1} - u^n recovered from two stored FP32 fields would carry
// the rounding of u (the 1001^2 workload at 500 steps: traces 1.5e-5 from
// the FP64 scheme in the plain form, 5.7e-7 in the difference form).
// ---------------------------------------------------------------------------
__device__ __forceinline__ float delta_update(float dc, float vv, float L, bool inband, float e, bool at_src,
                                              float qs) {
    float r;
    if (!inband) {
        r = fmaf(vv, L, dc);
        if (at_src) r += qs;
    } else {
        r = fmaf(vv, L, (1.f - e) * dc);
        if (at_src) r += qs;
        r *= __builtin_amdgcn_rcpf(1.f + e);   // hardware reciprocal (1 ulp), not a full division
    }
    return r;
}

// ---------------------------------------------------------------------------
// Per-step parameters of the single-shot forward kernels.
// ---------------------------------------------------------------------------
struct StepArgs {
    const float* __restrict__ ucur;  // u^n over the window (dense, x fastest)
    const float* dcur;               // d^n = u^n - u^{n-1} (may equal dnext: in-place update)
    float* dnext;                    // d^{n+1}
    float* unext;                    // u^{n+1} (never ucur: neighbours read u^n)
    const float* __restrict__ v;     // model v at the window origin
    long long ldv_y, ldv_z;          // model strides of v (row, plane)
    int nx, ny, nz;                  // window extent (ny = 1 in 2D)
    int tiles_x, tiles_y, ntiles;    // tile grid
    int zchunk;                      // 3D: planes per block
    Sponge sp;
    long long src;                   // source node (linear, window) or -1
    float q;                         // dt^2 / h^ndim
    const float* __restrict__ wavelet;
    int step;                        // n: the source sample s^n drives n -> n+1
    // receiver gather of u^n (= trace n-1), done by the first threads of the grid
    int nrec;
    const long long* __restrict__ rec_lin;
    float* __restrict__ trace_out;   // traces + (n-1)*nrec, or nullptr
    Weights w;
};

// Gradient parameter of the adjoint kernels: the gradient term at a point is
// f psi^{k+1} (W u^k) with f the derivative of the misfit's dependence on
// the chosen parameter, written through v = (c dt / h)^2:
//   velocity c:        2 / c      = gscale / sqrt(v),  gscale =  2 dt / h
//   slowness s = 1/c:  -2 c       = gscale * sqrt(v),  gscale = -2 h / dt
//   m = 1/c^2:         -c^2       = gscale * v,        gscale = -h^2 / dt^2
enum { GP_VELOCITY = 0, GP_SLOWNESS = 1, GP_M = 2 };

__device__ __forceinline__ float grad_factor(int gparam, float gscale, float v) {
    return gparam == GP_VELOCITY ? gscale * rsqrtf(v) : gparam == GP_SLOWNESS ? gscale * sqrtf(v) : gscale * v;
}

// Per-step parameters of the adjoint + gradient kernels.
struct AdjArgs {
    const float* __restrict__ pcur;  // psi^{k+1}
    const float* pprev;              // psi^{k+2} (may equal pnext)
    float* pnext;                    // psi^k
    const float* __restrict__ ufwd;  // u^k, paired with psi^{k+1} in the gradient
    const float* __restrict__ v;     // model v at the window origin
    float* __restrict__ grad;        // model gradient at the window origin (+=)
    float gscale;                    // see grad_factor
    int gparam;                      // GP_VELOCITY / GP_SLOWNESS / GP_M
    long long ldv_y, ldv_z;
    int nx, ny, nz;
    int tiles_x, tiles_y, ntiles;
    int zchunk;
    Sponge sp;
    int with_grad;                   // accumulate f psi^{k+1} (W u^k) into grad
    int with_update;                 // write psi^k
    Weights w;
};

// One shot of a batched launch (device memory, built by the host).  Each
// shot owns an arena of window-sized fields; kernels name fields by slot:
// slot s >= 0 is arena + s * npts;
// SLOT_INIT_DIFF / SLOT_INIT_CUR the caller's initial state d^0, u^0 (zeros
// when absent), SLOT_ZERO a field of zeros; SLOT_CKPT0 - i (i >= 0) is field
// i of the caller's checkpoint buffer (pair j = fields 2j (d), 2j+1 (u)).
enum { SLOT_ZERO = -3, SLOT_INIT_CUR = -2, SLOT_INIT_DIFF = -1, SLOT_CKPT0 = -16 };

struct BatchShot {
    float* arena;
    long long npts;                  // window points
    const float* v;                  // model v at the window origin
    long long ldv;                   // model row stride
    int nx, nz;                      // window
    int tiles_x, ntiles;             // tiles of this shot
    long long src;                   // window-linear source node
    const float* wavelet;
    int nrec;
    const long long* rec_lin;
    float* traces;
    const float* trace_adj;          // adjoint sources dJ/dtraces (adjoint calls)
    const float* init_diff;          // optional initial state d^0, u^0
    const float* init_cur;
    float* gacc;                     // window-shaped gradient accumulator (adjoint calls)
    float* ckpt;                     // caller's checkpoint fields, or nullptr
    int variant;                     // shape * 8 + (M - 1)
    Weights w;
};

__device__ __forceinline__ const float* slot_ptr(const BatchShot& s, int slot) {
    if (slot >= 0) return s.arena + (long long)slot * s.npts;
    if (slot == SLOT_INIT_DIFF) return s.init_diff;
    if (slot == SLOT_INIT_CUR) return s.init_cur;
    if (slot <= SLOT_CKPT0 && s.ckpt) return s.ckpt + (long long)(SLOT_CKPT0 - slot) * s.npts;
    return nullptr;
}

struct BatchArgs {
    const BatchShot* shots;
    const int2* jobs;                // (shot, tile within the shot) per block
    int njobs;
    int step;                        // forward: time step n (source sample, trace n-1)
    int f_ucur, f_dcur;              // forward: u^n, d^n slots
    int f_unext, f_dnext;            // u^{n+1}, d^{n+1} arena slots (f_dnext may equal f_dcur)
    int gather;                      // forward: write trace n-1 from u^n
    Sponge sp;
    float q;
};

struct BatchAdjArgs {
    const BatchShot* shots;
    const int2* jobs;
    int njobs;
    int f_pcur, f_pprev, f_pnext;    // psi^{k+1}, psi^{k+2}, psi^k slots
    int f_ufwd;                      // u^k slot (gradient pairing)
    int with_grad, with_update;
    float gscale;                    // see grad_factor
    int gparam;
    Sponge sp;
};

// one launch over the jobs of one stencil variant (false: not compiled)
bool launch_batch_adj2d(const BatchAdjArgs& a, int shape, int M, hipStream_t s);
// dst slot <- src slot for every shot (src SLOT_ZERO: fill with zeros; an
// absent initial state also reads as zeros); also used for gacc when dst is
// SLOT_GACC and for the caller's checkpoint fields (dst <= SLOT_CKPT0; shots
// without a checkpoint buffer are skipped)
enum { SLOT_GACC = -4 };
void launch_batch_copy(const BatchShot* shots, int nshots, long long max_npts, int dst, int src,
                       hipStream_t s);
// psi(x_r) += b v rho^{k-1}_r in slot f for every shot
void launch_batch_inject(const BatchShot* shots, int nshots, int max_nrec, int f, int k, Sponge sp,
                         hipStream_t s);
// trace n of every shot from slot f
void launch_batch_gather(const BatchShot* shots, int nshots, int max_nrec, int f, int n, hipStream_t s);
bool launch_batch2d(const BatchArgs& a, int shape, int M, int rows, hipStream_t s);
int batch_rows();   // rows per thread of the batched tiles (the adjoint's and the default)

// Launchers (one per translation unit).  Return false when the requested
// (shape, M, rows) combination was not compiled.
bool launch_fwd2d(const StepArgs& a, int shape, int M, int rows, hipStream_t s);
// 2D cross stencils marching along z (k_fwd2d_march, one row per thread):
// kBlock3 columns per block, tiles_x = ceil(nx / kBlock3), zchunk rows
bool launch_fwd2d_march(const StepArgs& a, int M, hipStream_t s);
bool launch_fwd3d(const StepArgs& a, int shape, int M, int rows, hipStream_t s);
bool launch_adj2d(const AdjArgs& a, int shape, int M, int rows, hipStream_t s);
bool launch_adj3d(const AdjArgs& a, int shape, int M, int rows, hipStream_t s);
bool have_fwd2d(int shape, int M, int rows);
bool have_fwd3d(int shape, int M, int rows);
bool have_adj3d(int shape, int M);
int adj_rows3d(int shape, int M, int fwd_rows);  // tile height the 3D adjoint runs with

// Small helper kernels (k_misc.hip).
// c_lim: largest stable Courant number (velocities above c_lim h / dt are flagged)
void launch_vprep(const float* vel, float* v, long long n, double dt_over_h, double c_lim, int* flags,
                  hipStream_t s);
void launch_fill(float* p, long long n, float val, hipStream_t s);
void launch_fill_i32(int* p, long long n, int val, hipStream_t s);
void launch_copy(float* dst, const float* src, long long n, hipStream_t s);
void launch_rec_index(const int* rec, int nrec, int ndim, int nx, int ny, int nz,
                      long long* lin, int* flags, hipStream_t s);
void launch_gather(const float* u, const long long* lin, int nrec, float* out, hipStream_t s);
// psi(x_r) += b(x_r) v(x_r) rho_r at every receiver (atomic: duplicates add up)
void launch_inject(float* psi, const long long* lin, int nrec, const float* rho, const float* v,
                   long long ldv_y, long long ldv_z, Sponge sp, int nx, int ny, int nz,
                   hipStream_t s);
void launch_check_finite(const float* p, long long n, int* flags, hipStream_t s);
// g[z*ldg + x] += a[z*nx + x] over an nx x nz window
void launch_accum2d(float* g, long long ldg, const float* a, int nx, int nz, hipStream_t s);

// flags[] slots in the workspace
enum { FLAG_BAD_REC = 0, FLAG_NONFINITE = 1, FLAG_BAD_VEL = 2, FLAG_UNSTABLE_VEL = 3, FLAG_COUNT = 4 };

// Dispersion metrics (k_disp.hip).  Half spectra are double2 [rc][nt/2+1],
// CWT fields double2 [rc][ns][nt].
void launch_rows_f64(const float* in, long long ld, double* out, int nt, int r0, int rc, hipStream_t s);
// (sum |e|, sum e^2, max |e|) of e = num - ref over an n[0] x n[1] x n[2]
// box of strided views into out[3] (device); partial holds 3 nblocks doubles
constexpr int kNormBlocks = 1024;
void launch_error_norms(const float* num, const long long* sn, const float* ref, const long long* sr,
                        const long long* n, double* partial, int nblocks, double* out, hipStream_t s);
void launch_gamma_dft(const void* A, const void* B, int nt, int rc, float* gamma, long long ldg, double* norm,
                      hipStream_t s);
void launch_cwt_spectra(const void* A, int nt, int rc, int ns, double dt, double omega0, void* W, hipStream_t s);
void launch_gamma_cwt(const void* Wn, const void* Wr, int nt, int rc, int ns, double* norm, hipStream_t s);

}  // namespace fdw
