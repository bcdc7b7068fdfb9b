// Host side of the C ABI declared in include/fdwave.h: argument validation,
// stencil registry (orbits, stability limit), workspace layout, kernel
// orchestration, HIP-graph cache, and the checkpointed adjoint.
#include "../../include/fdwave.h"

#include <hip/hip_runtime.h>
#include <rocfft/rocfft.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <list>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "fd_kernels.h"

using namespace fdw;

namespace {

// ---------------------------------------------------------------------------
// errors
// ---------------------------------------------------------------------------
thread_local std::string g_err;

int fail(int code, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return code;
}

#define HIP_OK(expr)                                                                   \
    do {                                                                               \
        hipError_t e_ = (expr);                                                        \
        if (e_ != hipSuccess)                                                          \
            return fail(FD_EDEVICE, "%s failed: %s", #expr, hipGetErrorString(e_));    \
    } while (0)

// ---------------------------------------------------------------------------
// orbits: one weight per orbit of the sign-flip / axis-permutation group
// (the point symmetry of Sec. 3.2).  Representative = absolute offsets in
// descending order; orbits in ascending lexicographic order.
// ---------------------------------------------------------------------------
struct Orbit {
    int rep[3];
    int count;
};

// Point sets of Sec. 4.1 (a >= b >= c >= 0 the sorted absolute offsets, c = 0
// in 2D): cross, rhombus (|x|+|z| <= M), square (max <= M), cross-rhombus
// (the cross of radius M plus the rhombus of size N) and cross-square (max
// <= M with the smaller offset <= N: a cross with arms N thick).
bool in_shape(int ndim, int shape, int M, int N, int a, int b, int c) {
    (void)ndim;
    switch (shape) {
        case FD_CROSS: return b == 0 && c == 0 && a <= M;
        case FD_RHOMBUS: return a + b + c <= M;
        case FD_SQUARE: return a <= M;
        case FD_CROSS_RHOMBUS: return (b == 0 && c == 0 && a <= M) || a + b + c <= N;
        case FD_CROSS_SQUARE: return a <= M && b <= N && c <= N;
    }
    return false;
}

std::vector<Orbit> make_orbits(int ndim, int shape, int M, int N) {
    std::vector<Orbit> out;
    for (int a = 0; a <= M; ++a)
        for (int b = 0; b <= a; ++b)
            for (int c = 0; c <= (ndim == 3 ? b : 0); ++c) {
                if (!in_shape(ndim, shape, M, N, a, b, c)) continue;
                Orbit o{{a, b, c}, 0};
                out.push_back(o);
            }
    // count points: enumerate the full box
    auto find = [&](int a, int b, int c) -> int {
        for (size_t i = 0; i < out.size(); ++i)
            if (out[i].rep[0] == a && out[i].rep[1] == b && out[i].rep[2] == c) return (int)i;
        return -1;
    };
    const int zr = ndim == 3 ? M : 0;
    for (int x = -M; x <= M; ++x)
        for (int y = -M; y <= M; ++y)
            for (int z = -zr; z <= zr; ++z) {
                int v[3] = {std::abs(x), std::abs(y), std::abs(z)};
                std::sort(v, v + 3, [](int p, int q) { return p > q; });
                int i = find(v[0], v[1], v[2]);
                if (i >= 0) out[i].count++;
            }
    return out;
}

// N-shapes are 2D (Sec. 4.1 defines them in 2D) with 0 <= N <= M; the basic
// shapes take N = 0.
bool valid_shape(int ndim, int shape, int M, int N) {
    if (!(ndim == 2 || ndim == 3) || M < 1 || M > FD_MAX_RADIUS) return false;
    if (shape >= FD_CROSS && shape <= FD_SQUARE) return N == 0;
    if (shape == FD_CROSS_RHOMBUS || shape == FD_CROSS_SQUARE) return ndim == 2 && N >= 0 && N <= M;
    return false;
}

// Kernel family of a shape: N-shapes without off-axis points are crosses,
// cross-rhombus(M, M) is the rhombus and cross-square(M, M) the square; the
// other N-shapes run the dense 2D kernels that take each column's extent
// from the stencil's mz table.
int kernel_shape(int shape, int M, int N) {
    switch (shape) {
        case FD_CROSS: return SH_CROSS;
        case FD_RHOMBUS: return SH_RHOMBUS;
        case FD_CROSS_RHOMBUS: return N <= 1 ? SH_CROSS : N == M ? SH_RHOMBUS : SH_NSHAPE;
        case FD_CROSS_SQUARE: return N == 0 ? SH_CROSS : N == M ? SH_SQUARE : SH_NSHAPE;
        default: return SH_SQUARE;
    }
}

// S(k) = sum_d w_d cos(k.d).  Summing an orbit over sign flips turns
// cos(k.d) into a product of cosines, so S is a sum over non-negative offset
// tuples of mult * w * prod_i cos(k_i |d_i|).
struct Symbol {
    int ndim, M;
    std::vector<double> coef;  // [(M+1)^ndim] weight * sign multiplicity per |offset| tuple
    double eval(const double* k) const {
        const int n = M + 1;
        double cx[FD_MAX_RADIUS + 1], cy[FD_MAX_RADIUS + 1], cz[FD_MAX_RADIUS + 1];
        for (int m = 0; m < n; ++m) {
            cx[m] = std::cos(k[0] * m);
            cy[m] = ndim == 3 ? std::cos(k[1] * m) : 1.0;
            cz[m] = std::cos(k[ndim - 1] * m);
        }
        double s = 0.0;
        if (ndim == 2) {
            for (int a = 0; a < n; ++a)
                for (int c = 0; c < n; ++c) s += coef[a * n + c] * cx[a] * cz[c];
        } else {
            for (int a = 0; a < n; ++a)
                for (int b = 0; b < n; ++b)
                    for (int c = 0; c < n; ++c) s += coef[(a * n + b) * n + c] * cx[a] * cy[b] * cz[c];
        }
        return s;
    }
};

Symbol make_symbol(int ndim, int shape, int M, int N, const std::vector<Orbit>& orbs,
                   const double* w) {
    Symbol S{ndim, M, {}};
    const int n = M + 1;
    S.coef.assign(ndim == 2 ? n * n : n * n * n, 0.0);
    for (int a = 0; a <= M; ++a)
        for (int b = 0; b <= (ndim == 3 ? M : 0); ++b)
            for (int c = 0; c <= M; ++c) {
                int v[3] = {a, b, c};
                if (ndim == 2) { v[1] = c; v[2] = 0; }
                int s[3] = {v[0], v[1], v[2]};
                std::sort(s, s + 3, [](int p, int q) { return p > q; });
                if (!in_shape(ndim, shape, M, N, s[0], s[1], s[2])) continue;
                int oi = -1;
                for (size_t i = 0; i < orbs.size(); ++i)
                    if (orbs[i].rep[0] == s[0] && orbs[i].rep[1] == s[1] && orbs[i].rep[2] == s[2])
                        oi = (int)i;
                int mult = (a ? 2 : 1) * (c ? 2 : 1) * (ndim == 3 && b ? 2 : 1);
                int idx = ndim == 2 ? a * n + c : (a * n + b) * n + c;
                S.coef[idx] += mult * w[oi];
            }
    return S;
}

// max over [0, pi]^ndim of -S and of S: dense sample, then a shrinking
// pattern search around the best sample.
void symbol_extrema(const Symbol& S, double* max_neg, double* max_pos) {
    const int ns = S.ndim == 2 ? 257 : 65;
    const double h = M_PI / (ns - 1);
    double best = -1e300, bpos = -1e300;
    double kbest[3] = {0, 0, 0};
    double k[3];
    const int ny = S.ndim == 3 ? ns : 1;
    for (int i = 0; i < ns; ++i)
        for (int j = 0; j < ny; ++j)
            for (int l = 0; l < ns; ++l) {
                k[0] = i * h;
                if (S.ndim == 3) { k[1] = j * h; k[2] = l * h; } else { k[1] = l * h; }
                const double s = S.eval(k);
                if (-s > best) { best = -s; std::memcpy(kbest, k, sizeof k); }
                bpos = std::max(bpos, s);
            }
    double step = h;
    for (int it = 0; it < 60; ++it) {
        bool improved = false;
        const int nd = S.ndim;
        int tot = nd == 2 ? 9 : 27;
        for (int t = 0; t < tot; ++t) {
            int d[3] = {t % 3 - 1, (t / 3) % 3 - 1, (t / 9) % 3 - 1};
            double kk[3];
            for (int q = 0; q < nd; ++q) kk[q] = std::min(M_PI, std::max(0.0, kbest[q] + step * d[q]));
            const double s = S.eval(kk);
            if (-s > best) { best = -s; std::memcpy(kbest, kk, sizeof kk); improved = true; }
        }
        if (!improved) step *= 0.5;
    }
    *max_neg = best;
    *max_pos = bpos;
}

// ---------------------------------------------------------------------------
// stencil registry
// ---------------------------------------------------------------------------
struct Stencil {
    int ndim, shape, M, nw;   // shape: kernel family (SH_CROSS / SH_RHOMBUS / SH_SQUARE / SH_NSHAPE)
    int ushape, N;            // the caller's shape and inner size
    std::vector<double> w64;
    Weights w32;
    double cfl;
    int rows, zchunk;
    int tsteps;   // single-shot forward: time steps per launch (1 or 2)
    int brows;    // batched 2D forward: rows per thread (0: 8 for dense shapes, 4 for crosses)
};

// rows per thread of a stencil's group in the forward steps of a batched call
int batch_forward_rows(const Stencil& st) {
    if (st.brows) return st.brows;
    return st.shape != SH_CROSS ? 8 : 4;
}

std::mutex g_mu;
std::vector<Stencil> g_stencils;

// Untuned defaults (the autotuner installs measured choices): 2D tiles of
// 64 x 16; 3D tiles of 64 x 8 (64 x 16 for crosses with M > 4).
int default_rows(int ndim, int shape, int M) {
    if (ndim == 2) return 4;
    if (shape == FD_CROSS) return 2;
    return 1;
}

bool get_stencil(int id, Stencil* out) {
    std::lock_guard<std::mutex> lk(g_mu);
    if (id < 0 || id >= (int)g_stencils.size()) return false;
    *out = g_stencils[id];
    return true;
}

// ---------------------------------------------------------------------------
// workspace layout
// ---------------------------------------------------------------------------
size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

struct ShotLayout {
    size_t arena;       // nslots window-sized fields: slot 0 = A, slot 1 = B, ...
    size_t rec;         // receiver indices
};
struct Layout {
    size_t flags, v;
    std::vector<ShotLayout> shots;
    int nslots;         // fields per shot arena
    // single-shot adjoint scratch (shared by all shots, sized for the largest window)
    size_t psiA, psiB, ckpt, seg;
    // batched calls: shot descriptors and the (shot, tile) work list
    size_t desc, jobs;
    long long njobs;
    size_t total;
};

// Call modes: forward, adjoint with segment checkpoints (K = segment
// length), adjoint with binomial checkpoints (K = snapshot count).
enum { MODE_FORWARD = 0, MODE_ADJ_SEGMENT = 1, MODE_ADJ_REVOLVE = 2 };

bool use_batch(const fd_grid* g, int nshots, int mode) {
    return nshots > 1 && g->ndim == 2 && !(g->flags & FD_NO_BATCH) && mode != MODE_ADJ_REVOLVE;
}

int shot_tiles2d(const fd_shot& s, int rows, int* tiles_x) {
    const int nx = (int)s.extent[0], nz = (int)s.extent[2];
    *tiles_x = (nx + kTileX - 1) / kTileX;
    return *tiles_x * ((nz + 4 * rows - 1) / (4 * rows));
}

long long window_points(const fd_shot& s, int ndim) {
    return s.extent[0] * (ndim == 3 ? s.extent[1] : 1) * s.extent[2];
}

// Slots of the batched adjoint arena (K = segment length, nseg segments):
// the forward state (u^n, u^{n+1}, d), checkpoint pairs (d^{jK}, u^{jK}), K
// segment fields for u and one for d, the two adjoint fields and the
// gradient accumulator.  With saved checkpoints (every shot passes
// fd_shot.ckpt) the pairs are read from the caller's buffer and take no
// arena slots.
struct AdjSlots {
    int nseg, K;
    bool saved = false;
    static constexpr int kU0 = 0, kU1 = 1, kD = 2;
    int nck() const { return saved ? 0 : 2 * nseg; }
    int ck(int j, int which) const { return saved ? SLOT_CKPT0 - (2 * j + which) : 3 + 2 * j + which; }
    int seg(int i) const { return 3 + nck() + i; }
    int dseg() const { return 3 + nck() + K; }
    int psiA() const { return dseg() + 1; }
    int psiB() const { return psiA() + 1; }
    int gacc() const { return psiA() + 2; }
    int count() const { return psiA() + 3; }
};

// shots passing saved checkpoints (fd_shot.ckpt)
int saved_count(const fd_shot* shots, int nshots) {
    int n = 0;
    for (int i = 0; i < nshots; ++i) n += shots[i].ckpt != nullptr;
    return n;
}

Layout make_layout(const fd_grid* g, const fd_shot* shots, int nshots, int mode, int K) {
    Layout L;
    size_t off = 0;
    L.flags = off;
    off += 256;
    const long long mpts = g->n[0] * (g->ndim == 3 ? g->n[1] : 1) * g->n[2];
    L.v = off;
    off = align256(off + sizeof(float) * (size_t)mpts);
    const bool batch = use_batch(g, nshots, mode);
    const int nseg = mode == MODE_ADJ_SEGMENT ? (g->nt + K - 1) / K : 0;
    // a forward arena holds u^n, u^{n+1} and d; the binomial adjoint keeps
    // its fields in the shared scratch below
    const int nsaved = mode == MODE_ADJ_SEGMENT ? saved_count(shots, nshots) : 0;
    L.nslots = (batch && mode == MODE_ADJ_SEGMENT) ? AdjSlots{nseg, K, nsaved == nshots}.count()
             : mode == MODE_ADJ_REVOLVE ? 0 : 3;
    long long wmax = 0;
    for (int i = 0; i < nshots; ++i) {
        const long long wp = window_points(shots[i], g->ndim);
        wmax = std::max(wmax, wp);
        ShotLayout sl;
        sl.arena = off;
        off = align256(off + sizeof(float) * (size_t)wp * (size_t)L.nslots);
        sl.rec = off;
        off = align256(off + sizeof(long long) * (size_t)std::max(shots[i].nrec, 0));
        L.shots.push_back(sl);
    }
    L.psiA = L.psiB = L.ckpt = L.seg = 0;
    if (mode != MODE_FORWARD && !batch) {
        // segments: nseg checkpoint pairs (none when every shot brings its
        // own), K segment fields for u and one for d; binomial: K snapshot
        // pairs, three working fields (the current state and the next u)
        // and one of zeros for an absent initial state
        const size_t nck = mode == MODE_ADJ_SEGMENT ? (nsaved == nshots ? 0 : (size_t)nseg) : (size_t)K;
        const size_t nsegf = mode == MODE_ADJ_SEGMENT ? (size_t)K + 1 : 4;
        L.psiA = off;
        off = align256(off + sizeof(float) * (size_t)wmax);
        L.psiB = off;
        off = align256(off + sizeof(float) * (size_t)wmax);
        L.ckpt = off;
        off = align256(off + sizeof(float) * (size_t)wmax * 2 * nck);
        L.seg = off;
        off = align256(off + sizeof(float) * (size_t)wmax * nsegf);
    }
    L.desc = L.jobs = 0;
    L.njobs = 0;
    if (batch) {
        int tx;
        for (int i = 0; i < nshots; ++i) L.njobs += shot_tiles2d(shots[i], batch_rows(), &tx);
        L.desc = off;
        off = align256(off + sizeof(BatchShot) * (size_t)nshots);
        L.jobs = off;
        off = align256(off + sizeof(int2) * (size_t)L.njobs);
    }
    L.total = off;
    return L;
}

// ---------------------------------------------------------------------------
// validation
// ---------------------------------------------------------------------------
int check_grid(const fd_grid* g) {
    if (!g) return fail(FD_EINVAL, "grid is NULL");
    if (g->ndim != 2 && g->ndim != 3) return fail(FD_EINVAL, "ndim must be 2 or 3 (got %d)", g->ndim);
    if (g->nt < 1) return fail(FD_EINVAL, "nt must be >= 1 (got %d)", g->nt);
    if (g->flags & ~(FD_NO_GRAPH | FD_NO_BATCH))
        return fail(FD_EINVAL, "unknown flags 0x%x", (unsigned)g->flags);
    if (g->n[0] < 1 || g->n[2] < 1 || (g->ndim == 3 && g->n[1] < 1))
        return fail(FD_EINVAL, "model extents must be >= 1");
    if (g->ndim == 2 && g->n[1] != 1) return fail(FD_EINVAL, "2D models need n[1] == 1");
    if (g->n[0] > (1LL << 30) || g->n[1] > (1LL << 30) || g->n[2] > (1LL << 30))
        return fail(FD_EINVAL, "model extent too large");
    if (!(g->h > 0) || !(g->dt > 0) || !std::isfinite(g->h) || !std::isfinite(g->dt))
        return fail(FD_EINVAL, "h and dt must be positive and finite");
    if (g->nb < 0) return fail(FD_EINVAL, "nb must be >= 0");
    if (!(g->eta_max >= 0) || !std::isfinite(g->eta_max)) return fail(FD_EINVAL, "eta_max must be >= 0");
    if (!(g->vmax > 0) || !std::isfinite(g->vmax)) return fail(FD_EINVAL, "vmax must be positive");
    return FD_OK;
}

int check_shot(const fd_grid* g, const fd_shot& s, int i, bool adjoint, Stencil* st) {
    if (!get_stencil(s.stencil_id, st)) return fail(FD_EINVAL, "shot %d: unknown stencil id %d", i, s.stencil_id);
    if (st->ndim != g->ndim) return fail(FD_EINVAL, "shot %d: stencil is %dD, grid is %dD", i, st->ndim, g->ndim);
    for (int a = 0; a < 3; ++a) {
        if (g->ndim == 2 && a == 1) {
            if (s.origin[1] != 0 || s.extent[1] != 1) return fail(FD_EINVAL, "shot %d: 2D windows need origin[1]=0, extent[1]=1", i);
            continue;
        }
        if (s.extent[a] < 1 || s.origin[a] < 0 || s.origin[a] + s.extent[a] > g->n[a])
            return fail(FD_EINVAL, "shot %d: window axis %d [%lld, %lld) outside the model [0, %lld)", i, a,
                        s.origin[a], s.origin[a] + s.extent[a], g->n[a]);
    }
    for (int a = 0; a < 3; ++a) {
        if (g->ndim == 2 && a == 1) continue;
        if (s.src[a] < 0 || s.src[a] >= s.extent[a])
            return fail(FD_EINVAL, "shot %d: source coordinate %d = %d outside the window", i, a, s.src[a]);
    }
    if (!s.wavelet) return fail(FD_EINVAL, "shot %d: wavelet is NULL", i);
    if (s.nrec < 0) return fail(FD_EINVAL, "shot %d: nrec < 0", i);
    if (s.nrec > 0 && (!s.rec || !s.traces)) return fail(FD_EINVAL, "shot %d: rec/traces NULL with nrec > 0", i);
    if (adjoint && s.nrec > 0 && !s.trace_adj) return fail(FD_EINVAL, "shot %d: trace_adj is NULL", i);
    const double courant = g->vmax * g->dt / g->h;
    if (courant > st->cfl)
        return fail(FD_EUNSTABLE, "shot %d: Courant number vmax*dt/h = %.6g exceeds the stencil's limit %.6g",
                    i, courant, st->cfl);
    const bool have = g->ndim == 2 ? have_fwd2d(st->shape, st->M, st->rows)
                                   : have_fwd3d(st->shape, st->M, st->rows);
    if (!have)
        return fail(FD_EUNSUPPORTED, "shot %d: no compiled %dD kernel for shape %d, M = %d, rows = %d", i,
                    g->ndim, st->shape, st->M, st->rows);
    if (adjoint && g->ndim == 3 && !have_adj3d(st->shape, st->M))
        return fail(FD_EUNSUPPORTED, "shot %d: no compiled 3D adjoint kernel for shape %d, M = %d", i,
                    st->shape, st->M);
    return FD_OK;
}

// ---------------------------------------------------------------------------
// graph cache: one instantiated graph per distinct call signature
// ---------------------------------------------------------------------------
int g_graph_fallbacks = 0;

struct GraphCache {
    std::mutex mu;
    struct Entry {
        std::vector<uint64_t> key;
        std::vector<hipGraphExec_t> execs;
        void* pinned = nullptr;     // immutable host copy of the call's blob
        size_t pinned_bytes = 0;
    };
    std::list<Entry> lru;
    std::map<int, hipStream_t> capture_streams;
    static constexpr size_t kCap = 24;
} g_graphs;

void key_push(std::vector<uint64_t>& k, const void* p, size_t n) {
    const unsigned char* c = (const unsigned char*)p;
    for (size_t i = 0; i < n; i += 8) {
        uint64_t w = 0;
        std::memcpy(&w, c + i, std::min<size_t>(8, n - i));
        k.push_back(w);
    }
}

// Streams and events for independent work that may run concurrently
// (per device, library-owned, default priority).  Captured into a graph, the
// fork / join dependencies become graph edges and the branches run on
// separate hardware queues; without capture they are real cross-stream waits.
constexpr int kBranches = 4;

struct Branches {
    hipStream_t s[kBranches];
    hipEvent_t fork;
    hipEvent_t join[kBranches];
};
std::map<int, Branches> g_branches;
std::mutex g_branch_mu;   // held while a call enqueues its work

// Created outside any capture (called before a capture begins).
int get_branches(Branches** out) {
    std::lock_guard<std::mutex> lk(g_branch_mu);
    int dev = 0;
    HIP_OK(hipGetDevice(&dev));
    auto it = g_branches.find(dev);
    if (it == g_branches.end()) {
        Branches b;
        for (int i = 0; i < kBranches; ++i) {
            HIP_OK(hipStreamCreateWithFlags(&b.s[i], hipStreamNonBlocking));
            HIP_OK(hipEventCreateWithFlags(&b.join[i], hipEventDisableTiming));
        }
        HIP_OK(hipEventCreateWithFlags(&b.fork, hipEventDisableTiming));
        it = g_branches.emplace(dev, b).first;
    }
    *out = &it->second;
    return FD_OK;
}

// Splits captured work into graphs of bounded size: HIP graph capture and
// instantiation cost grow with the node count, and a multi-shot adjoint
// would otherwise become one graph of ~10^5 nodes.  In direct mode (no
// capture) cuts do nothing.  Work may be forked onto up to kBranches branch
// streams (on(b)); a cut joins the branches, ends the graph and forks again.
struct Recorder {
    bool capturing = false;
    hipStream_t stream = nullptr;
    std::vector<hipGraphExec_t> execs;
    int nodes = 0;
    int err = FD_OK;
    Branches* br = nullptr;
    int nbr = 0;          // forked branches (0: everything on `stream`)
    static constexpr int kMaxNodes = 2048;

    int active = -1;      // branch that per-shot enqueue functions use (-1: `stream`)

    hipStream_t on(int b) const { return nbr > 0 ? br->s[b % nbr] : stream; }
    hipStream_t cur() const { return active >= 0 ? on(active) : stream; }
    void launched(int n = 1) {
        nodes += n;
        if (nodes >= kMaxNodes) cut();
    }
    void check(hipError_t e) {
        if (e != hipSuccess && err == FD_OK) err = fail(FD_EDEVICE, "stream fork/join failed: %s", hipGetErrorString(e));
    }
    // branches 0..n-1 start after everything queued so far on `stream`
    void fork(int n) {
        n = std::min(n, kBranches);
        if (n <= 1 || !br) return;
        check(hipEventRecord(br->fork, stream));
        for (int b = 0; b < n; ++b) check(hipStreamWaitEvent(br->s[b], br->fork, 0));
        nbr = n;
    }
    // `stream` continues after everything queued on the branches
    void join() {
        if (nbr == 0) return;
        for (int b = 0; b < nbr; ++b) {
            check(hipEventRecord(br->join[b], br->s[b]));
            check(hipStreamWaitEvent(stream, br->join[b], 0));
        }
        nbr = 0;
    }
    // End the current capture, keep its graph, and start capturing again.
    // After a failure the remaining work is still captured (and later
    // discarded) so that nothing runs outside the caller's stream order.
    void cut() {
        if (!capturing || nodes == 0) return;
        const int forked = nbr;
        join();
        hipGraph_t graph = nullptr;
        hipError_t e = hipStreamEndCapture(stream, &graph);
        hipGraphExec_t exec = nullptr;
        if (e == hipSuccess && err == FD_OK) e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
        if (graph) hipGraphDestroy(graph);
        if (exec) execs.push_back(exec);
        if (e != hipSuccess && err == FD_OK)
            err = fail(FD_EDEVICE, "graph capture failed: %s", hipGetErrorString(e));
        nodes = 0;
        e = hipStreamBeginCapture(stream, hipStreamCaptureModeThreadLocal);
        if (e != hipSuccess) {
            if (err == FD_OK) err = fail(FD_EDEVICE, "graph capture failed: %s", hipGetErrorString(e));
            capturing = false;
            return;
        }
        fork(forked);
    }
};

// ---------------------------------------------------------------------------
// per-call context and the enqueued work
// ---------------------------------------------------------------------------
struct ShotCtx {
    const fd_shot* s;
    Stencil st;
    int nx, ny, nz;
    long long npts;
    const float* v;   // model v at the window origin
    float* bufA;
    float* bufB;
    long long* rec;
    long long src;
};

struct CallCtx {
    const fd_grid* g;
    const float* vel;
    int nshots;
    std::vector<ShotCtx> shots;
    Layout L;
    char* ws;
    int* flags;
    float* vfield;
    long long ldv_y, ldv_z;
    Sponge sp;
    float q;
    double c_lim;   // smallest stability limit over the call's stencils
    // adjoint: K = segment length (segments) or snapshot count (binomial);
    // gparam = GP_* parameter of the gradient
    int K;
    int gparam = GP_VELOCITY;
    float* grad;
    // host-built data uploaded to the workspace before the work runs
    std::vector<unsigned char> blob;
    size_t blob_off = 0;
    // batched calls: shots grouped by stencil variant (contiguous in the
    // descriptor array and in the work list), each group on a branch
    struct Group {
        int shape, M;
        int rows;                 // rows per thread of the group's tiles
        int d0, dn;               // descriptor range
        long long job0, njobs;    // work-list range
        long long maxn;           // largest window of the group
        int maxrec;
        int branch;
    };
    std::vector<Group> groups;
    int nbranch = 1;
};

// offset of a window origin in model-sized arrays
long long model_offset(const CallCtx& c, const fd_shot& s) {
    return s.origin[2] * c.ldv_z + s.origin[1] * c.ldv_y + s.origin[0];
}

void fill_tiles(StepArgs& a, int ndim, int rows, int zchunk) {
    if (ndim == 2 && rows == 1) {   // marching kernel: kBlock3 columns by zchunk rows
        a.tiles_x = (a.nx + kBlock3 - 1) / kBlock3;
        a.tiles_y = 1;
        a.ntiles = a.tiles_x * ((a.nz + zchunk - 1) / zchunk);
        a.zchunk = zchunk;
    } else if (ndim == 2) {
        a.tiles_x = (a.nx + kTileX - 1) / kTileX;
        a.tiles_y = 1;
        const int tz = (a.nz + 4 * rows - 1) / (4 * rows);
        a.ntiles = a.tiles_x * tz;
        a.zchunk = 0;
    } else {
        a.tiles_x = (a.nx + kTileX - 1) / kTileX;
        a.tiles_y = (a.ny + kWaves3 * rows - 1) / (kWaves3 * rows);
        const int tz = (a.nz + zchunk - 1) / zchunk;
        a.ntiles = a.tiles_x * a.tiles_y * tz;
        a.zchunk = zchunk;
    }
}

StepArgs base_step(const CallCtx& c, const ShotCtx& s) {
    StepArgs a;
    std::memset(&a, 0, sizeof a);
    a.v = s.v;
    a.ldv_y = c.ldv_y;
    a.ldv_z = c.ldv_z;
    a.nx = s.nx;
    a.ny = s.ny;
    a.nz = s.nz;
    fill_tiles(a, c.g->ndim, s.st.rows, s.st.zchunk);
    a.sp = c.sp;
    a.src = s.src;
    a.q = c.q;
    a.wavelet = s.s->wavelet;
    a.nrec = s.s->nrec;
    a.rec_lin = s.rec;
    a.w = s.st.w32;
    return a;
}

bool launch_step(const CallCtx& c, const ShotCtx& s, const StepArgs& a, hipStream_t st) {
    if (c.g->ndim == 2) return launch_fwd2d(a, s.st.shape, s.st.M, s.st.rows, st);
    return launch_fwd3d(a, s.st.shape, s.st.M, s.st.rows, st);
}

// Fields of a shot's forward arena: two buffers for u (u^{n+1} never
// overwrites u^n, which neighbouring points read in the same launch) and
// one for d, updated in place.
float* arena_u(const ShotCtx& s, int i) { return s.bufA + (size_t)i * s.npts; }
float* arena_d(const ShotCtx& s) { return s.bufA + 2 * (size_t)s.npts; }

// Initial state (d^0, u^0) into the arena: the caller's, or zeros.
void load_initial_state(const ShotCtx& s, float* u0, float* d0, hipStream_t st, Recorder& R) {
    const long long n = s.npts;
    if (s.s->init_cur) launch_copy(u0, s.s->init_cur, n, st); else launch_fill(u0, n, 0.f, st);
    if (s.s->init_diff) launch_copy(d0, s.s->init_diff, n, st); else launch_fill(d0, n, 0.f, st);
    R.launched(2);
}

// forward run of one shot on the state (u^n, d^n).  With ckpt != nullptr,
// pair j receives (d^{jK}, u^{jK}) for every segment start jK; with seg !=
// nullptr too, the steps of the last segment [tail, nt) write u^{n+1} out of
// place into seg[n - tail] (so the adjoint needs no recompute for that
// segment).
int enqueue_forward_shot(const CallCtx& c, const ShotCtx& s, float* ckpt, int K, float* seg,
                         Recorder& R) {
    hipStream_t st = R.cur();
    const long long n = s.npts;
    const int nt = c.g->nt;
    float* U[2] = {arena_u(s, 0), arena_u(s, 1)};
    float* D = arena_d(s);
    load_initial_state(s, U[0], D, st, R);
    launch_rec_index(s.s->rec, s.s->nrec, c.g->ndim, s.nx, s.ny, s.nz, s.rec, c.flags, st);
    R.launched();
    const int tail = (ckpt && seg) ? ((nt - 1) / K) * K : nt;
    if (ckpt) {
        launch_copy(ckpt, D, n, st);
        launch_copy(ckpt + n, U[0], n, st);
        R.launched(2);
    }
    StepArgs a = base_step(c, s);
    a.dcur = a.dnext = D;
    int cur = 0;
    const float* last = U[0];
    for (int step = 0; step < nt; ++step) {
        a.step = step;
        a.trace_out = (step > 0 && s.s->nrec > 0) ? s.s->traces + (size_t)(step - 1) * s.s->nrec : nullptr;
        if (step < tail) {
            a.ucur = U[cur];
            a.unext = U[cur ^ 1];
        } else {
            const int i = step - tail;
            a.ucur = i == 0 ? U[cur] : seg + (size_t)(i - 1) * n;
            a.unext = seg + (size_t)i * n;
        }
        if (!launch_step(c, s, a, st)) return fail(FD_EUNSUPPORTED, "kernel not compiled");
        R.launched();
        last = a.unext;
        if (step < tail) {
            cur ^= 1;
            if (ckpt && (step + 1) % K == 0 && step + 1 < nt) {
                float* pair = ckpt + (size_t)((step + 1) / K) * 2 * n;
                launch_copy(pair, D, n, st);
                launch_copy(pair + n, U[cur], n, st);
                R.launched(2);
            }
        }
    }
    if (s.s->nrec > 0)
        launch_gather(last, s.rec, s.s->nrec, s.s->traces + (size_t)(nt - 1) * s.s->nrec, st);
    if (s.s->final_diff) launch_copy(s.s->final_diff, D, n, st);
    if (s.s->final_cur) launch_copy(s.s->final_cur, last, n, st);
    if (c.g->check_finite && s.s->nrec > 0)
        launch_check_finite(s.s->traces, (long long)nt * s.s->nrec, c.flags, st);
    R.launched(4);
    return R.err;
}

// the 2D marching forward kernel (rows 1) has no adjoint twin: the 2D
// adjoint then runs its tiled kernel at 4 rows per thread
int adj_rows(const CallCtx& c, const ShotCtx& s) {
    return c.g->ndim == 3 ? adj_rows3d(s.st.shape, s.st.M, s.st.rows) : (s.st.rows == 1 ? 4 : s.st.rows);
}

// gscale of grad_factor for the call's gradient parameter
float grad_scale(const CallCtx& c) {
    const double dt = c.g->dt, h = c.g->h;
    if (c.gparam == GP_SLOWNESS) return (float)(-2.0 * h / dt);
    if (c.gparam == GP_M) return (float)(-(h * h) / (dt * dt));
    return (float)(2.0 * dt / h);
}

AdjArgs base_adj(const CallCtx& c, const ShotCtx& s) {
    AdjArgs a;
    std::memset(&a, 0, sizeof a);
    a.v = s.v;
    a.grad = c.grad + model_offset(c, *s.s);
    a.gscale = grad_scale(c);
    a.gparam = c.gparam;
    a.ldv_y = c.ldv_y;
    a.ldv_z = c.ldv_z;
    a.nx = s.nx;
    a.ny = s.ny;
    a.nz = s.nz;
    StepArgs t;
    t.nx = s.nx; t.ny = s.ny; t.nz = s.nz;
    // the 3D adjoint runs taller tiles than the forward; chunks of at most 256
    // planes keep its block count up (512^3, 4 rows: 256 blocks at 256 planes,
    // 128 at 512, i.e. half the CUs idle)
    fill_tiles(t, c.g->ndim, adj_rows(c, s), c.g->ndim == 3 ? std::min(s.st.zchunk, 256) : s.st.zchunk);
    a.tiles_x = t.tiles_x;
    a.tiles_y = t.tiles_y;
    a.ntiles = t.ntiles;
    a.zchunk = t.zchunk;
    a.sp = c.sp;
    a.w = s.st.w32;
    return a;
}

bool launch_adj(const CallCtx& c, const ShotCtx& s, const AdjArgs& a, hipStream_t st) {
    if (c.g->ndim == 2) return launch_adj2d(a, s.st.shape, s.st.M, adj_rows(c, s), st);
    return launch_adj3d(a, s.st.shape, s.st.M, adj_rows(c, s), st);
}

// forward with checkpoints, then segment-wise recompute + adjoint, one shot
int enqueue_adjoint_shot(const CallCtx& c, const ShotCtx& s, Recorder& R) {
    hipStream_t st = R.stream;
    const int nt = c.g->nt, K = c.K;
    const long long n = s.npts;
    // saved checkpoints: the forward pass ran in an earlier fd_forward call
    const bool saved = s.s->ckpt != nullptr;
    float* ckpt = saved ? s.s->ckpt : (float*)(c.ws + c.L.ckpt);
    float* seg = (float*)(c.ws + c.L.seg);
    float* pa = (float*)(c.ws + c.L.psiA);
    float* pb = (float*)(c.ws + c.L.psiB);
    if (saved) {
        launch_rec_index(s.s->rec, s.s->nrec, c.g->ndim, s.nx, s.ny, s.nz, s.rec, c.flags, st);
        R.launched();
    } else {
        int rc = enqueue_forward_shot(c, s, ckpt, K, seg, R);
        if (rc) return rc;
        R.cut();
    }
    launch_fill(pa, n, 0.f, st);   // psi^{nt+1}
    launch_fill(pb, n, 0.f, st);   // psi^{nt+2}
    float* pcur = pa;
    float* pprev = pb;
    const int nseg = (nt + K - 1) / K;
    StepArgs f = base_step(c, s);
    f.trace_out = nullptr;
    AdjArgs a = base_adj(c, s);
    float* dseg = seg + (size_t)K * n;   // d during a segment's recompute
    for (int j = nseg - 1; j >= 0; --j) {
        const int s0 = j * K, e0 = std::min(nt, s0 + K);
        const float* ck_d = ckpt + (size_t)j * 2 * n;
        const float* ck_u = ck_d + n;
        // recompute u^{s0+1} .. u^{e0} into seg[0 .. e0-s0-1] from the pair
        // (d^{s0}, u^{s0}) (the last segment is already there when this call
        // ran the forward pass); d goes to dseg, in place after the first step
        for (int step = s0; step < e0 && (j < nseg - 1 || saved); ++step) {
            const int i = step - s0;
            f.ucur = i == 0 ? ck_u : seg + (size_t)(i - 1) * n;
            f.dcur = i == 0 ? ck_d : dseg;
            f.dnext = dseg;
            f.unext = seg + (size_t)i * n;
            f.step = step;
            if (!launch_step(c, s, f, st)) return fail(FD_EUNSUPPORTED, "kernel not compiled");
            R.launched();
        }
        // adjoint iterations k = e0 .. s0+1: psi^k from psi^{k+1}, psi^{k+2};
        // gradient term (2/c) psi^{k+1} (W u^k) for k < nt
        for (int k = e0; k > s0; --k) {
            a.pcur = pcur;
            a.pprev = pprev;
            a.pnext = pprev;
            a.ufwd = seg + (size_t)(k - s0 - 1) * n;
            a.with_grad = k < nt;
            a.with_update = 1;
            if (!launch_adj(c, s, a, st)) return fail(FD_EUNSUPPORTED, "adjoint kernel not compiled");
            if (s.s->nrec > 0)
                launch_inject(pprev, s.rec, s.s->nrec, s.s->trace_adj + (size_t)(k - 1) * s.s->nrec, s.v,
                              c.ldv_y, c.ldv_z, c.sp, s.nx, s.ny, s.nz, st);
            std::swap(pcur, pprev);
            R.launched(2);
        }
        R.cut();
    }
    // last gradient term (2/c) psi^1 (W u^0): non-zero only with initial data
    if (s.s->init_cur) {
        a.pcur = pcur;
        a.pprev = pprev;
        a.pnext = pprev;
        a.ufwd = s.s->init_cur;
        a.with_grad = 1;
        a.with_update = 0;
        if (!launch_adj(c, s, a, st)) return fail(FD_EUNSUPPORTED, "adjoint kernel not compiled");
        R.launched();
    }
    return R.err;
}

// ---------------------------------------------------------------------------
// binomial checkpointing (Griewank & Walther, ACM TOMS 26, 2000: "revolve")
// ---------------------------------------------------------------------------
// The adjoint iteration k (k = nt .. 1) needs u^k, i.e. the forward state
// S_k = (d^k, u^k) (difference form, d^k = u^k - u^{k-1}); S_0 is the
// initial data.  With s snapshot slots, the
// least number of forward steps that serves every iteration is, for
// l = nt + 1 and r = s + 1 stored states (S_0 included), t l - C(r+t, r+1)
// with t the least integer such that C(r+t, r) >= l.  The plan reaches it by
// the binomial split: advance S_a -> S_{a+m}, store it, serve (a+m, b] with
// one slot fewer, run iteration a+m on the stored state, then serve
// (a, a+m-1] from S_a with every slot; m minimises
// m + cost(b-a-m, s-1) + cost(m-1, s), a convex function of m.
struct RevolvePlanner {
    int nsnap;
    std::vector<int> ops;   // (op, arg) pairs, FD_OP_*

    static long long cost(long long L, int s) {
        if (L <= 0) return 0;
        const long long l = L + 1;
        const unsigned long long r = (unsigned long long)s + 1;
        // b = C(r+t, r), grown one t at a time (exact: C(n+1, r) = C(n, r) (n+1) / (n+1-r))
        unsigned long long b = 1, t = 0;
        while (b < (unsigned long long)l) {
            ++t;
            b = (unsigned long long)((unsigned __int128)b * (r + t) / t);
        }
        // C(r+t, r+1) = C(r+t, r) t / (r+1)
        const unsigned long long b1 = (unsigned long long)((unsigned __int128)b * t / (r + 1));
        return (long long)(t * (unsigned long long)l - b1);
    }
    void emit(int op, int arg) {
        ops.push_back(op);
        ops.push_back(arg);
    }
    // serve iterations b .. a+1; S_a is in slot sa (-1: the initial data);
    // slots >= next are free; cur: whether the current state is S_a
    void serve(int a, int b, int sa, int next, bool cur) {
        while (b > a) {
            const int l = b - a, k = nsnap - next;
            if (!cur) emit(FD_OP_RESTORE, sa);
            cur = false;
            if (l == 1 || k == 0) {   // advance to b, iteration b, restart from S_a
                emit(FD_OP_ADVANCE, b);
                emit(FD_OP_ADJOINT, b);
                --b;
                continue;
            }
            int best = l;
            long long bc = cost(l - 1, k) + l;
            for (int m = 1; m < l; ++m) {
                const long long c = m + cost(l - m, k - 1) + cost(m - 1, k);
                if (c < bc) {
                    bc = c;
                    best = m;
                }
            }
            if (best == l) {
                emit(FD_OP_ADVANCE, b);
                emit(FD_OP_ADJOINT, b);
                --b;
                continue;
            }
            emit(FD_OP_ADVANCE, a + best);
            emit(FD_OP_STORE, next);
            serve(a + best, b, next, next + 1, true);
            emit(FD_OP_RESTORE, next);
            emit(FD_OP_ADJOINT, a + best);
            b = a + best - 1;
        }
    }
    long long plan(int nt, int s) {
        nsnap = s;
        ops.clear();
        serve(0, nt, -1, 0, true);
        long long steps = 0, cur = 0;
        std::vector<long long> slot(std::max(s, 1), 0);
        for (size_t i = 0; i < ops.size(); i += 2) {
            if (ops[i] == FD_OP_ADVANCE) {
                steps += ops[i + 1] - cur;
                cur = ops[i + 1];
            } else if (ops[i] == FD_OP_STORE) {
                slot[ops[i + 1]] = cur;
            } else if (ops[i] == FD_OP_RESTORE) {
                cur = ops[i + 1] < 0 ? 0 : slot[ops[i + 1]];
            }
        }
        return steps;
    }
};

// Adjoint of one shot under a binomial plan.  The forward fields live in a
// pool of 2 nsnap + 2 window fields (the snapshot region and W0, W1);
// a snapshot is a pair of references into the pool (or to the initial data),
// so STORE copies nothing.  A step writes u^{k+1} over u^{k-1} when no live
// snapshot references that field, else into a pool field referenced by
// neither a snapshot nor the current state: at most 2 nsnap fields are
// referenced by snapshots and one more by the current state, so one is
// always free.  Traces are written the first time a step runs (the first
// pass runs every step in order).
int enqueue_adjoint_revolve(const CallCtx& c, const ShotCtx& s, Recorder& R) {
    hipStream_t st = R.stream;
    const int nt = c.g->nt, nrec = s.s->nrec, nsnap = c.K;
    const long long n = s.npts;
    float* ckpt = (float*)(c.ws + c.L.ckpt);
    float* W0 = (float*)(c.ws + c.L.seg);
    float* Z = W0 + 3 * n;
    float* pa = (float*)(c.ws + c.L.psiA);
    float* pb = (float*)(c.ws + c.L.psiB);
    RevolvePlanner planner;
    planner.plan(nt, nsnap);
    const std::vector<int>& ops = planner.ops;

    // pool field i: the snapshot region for i < 2 nsnap, then W0, W1, W2.
    // A state is (U, D) = (u^k, d^k); snapshots reference pool fields
    // (pins), nothing is copied.  A step writes u^{k+1} into a free field and
    // d^{k+1} over d^k unless d^k is referenced.  At most 2 nsnap + 2 fields
    // are referenced (the snapshots and an unreferenced current state, whose
    // d is then updated in place), so a step always finds the fields it needs.
    const int npool = 2 * nsnap + 3;
    auto field = [&](int i) { return i < 2 * nsnap ? ckpt + (size_t)i * n : W0 + (size_t)(i - 2 * nsnap) * n; };
    auto index = [&](const float* f) -> int {
        if (nsnap > 0 && f >= ckpt && f < ckpt + (size_t)2 * nsnap * n) return (int)((f - ckpt) / n);
        for (int w = 0; w < 3; ++w)
            if (f == W0 + (size_t)w * n) return 2 * nsnap + w;
        return -1;   // initial data or the zero field
    };
    std::vector<int> pins(npool, 0);
    std::vector<const float*> snap_u(std::max(nsnap, 1), nullptr), snap_d(std::max(nsnap, 1), nullptr);
    std::vector<int> snap_step(std::max(nsnap, 1), 0);
    auto pin = [&](const float* f, int d) {
        const int i = index(f);
        if (i >= 0) pins[i] += d;
    };

    launch_rec_index(s.s->rec, nrec, c.g->ndim, s.nx, s.ny, s.nz, s.rec, c.flags, st);
    R.launched();
    if (!s.s->init_diff || !s.s->init_cur) {
        launch_fill(Z, n, 0.f, st);
        R.launched();
    }
    const float* init_u = s.s->init_cur ? s.s->init_cur : Z;
    const float* init_d = s.s->init_diff ? s.s->init_diff : Z;
    const float* U = init_u;
    const float* D = init_d;
    int cur = 0, hi = 0;
    StepArgs f = base_step(c, s);
    launch_fill(pa, n, 0.f, st);   // psi^{nt+1}
    launch_fill(pb, n, 0.f, st);   // psi^{nt+2}
    R.launched(2);
    float* pcur = pa;
    float* pprev = pb;
    AdjArgs a = base_adj(c, s);
    for (size_t i = 0; i < ops.size(); i += 2) {
        const int op = ops[i], arg = ops[i + 1];
        if (op == FD_OP_ADVANCE) {
            while (cur < arg) {
                const int iu = index(U), id = index(D);
                auto free_field = [&](int except) {
                    for (int j = 0; j < npool; ++j)
                        if (pins[j] == 0 && j != iu && j != id && j != except) return j;
                    return -1;
                };
                const int ju = free_field(-1);
                const int jd = (id >= 0 && pins[id] == 0) ? id : free_field(ju);
                if (ju < 0 || jd < 0) return fail(FD_EDEVICE, "binomial adjoint: no free field (internal error)");
                float* Un = field(ju);
                float* Dn = field(jd);
                f.ucur = U;
                f.dcur = D;
                f.dnext = Dn;
                f.unext = Un;
                f.step = cur;
                f.trace_out = (cur >= hi && cur >= 1 && nrec > 0) ? s.s->traces + (size_t)(cur - 1) * nrec : nullptr;
                if (!launch_step(c, s, f, st)) return fail(FD_EUNSUPPORTED, "kernel not compiled");
                R.launched();
                U = Un;
                D = Dn;
                ++cur;
                if (cur > hi) {
                    hi = cur;
                    if (hi == nt) {   // trace nt-1 <- u^nt; final state
                        if (nrec > 0) launch_gather(U, s.rec, nrec, s.s->traces + (size_t)(nt - 1) * nrec, st);
                        if (s.s->final_diff) launch_copy(s.s->final_diff, D, n, st);
                        if (s.s->final_cur) launch_copy(s.s->final_cur, U, n, st);
                        R.launched(3);
                    }
                }
            }
        } else if (op == FD_OP_STORE) {
            if (snap_u[arg]) {
                pin(snap_u[arg], -1);
                pin(snap_d[arg], -1);
            }
            snap_u[arg] = U;
            snap_d[arg] = D;
            snap_step[arg] = cur;
            pin(U, 1);
            pin(D, 1);
        } else if (op == FD_OP_RESTORE) {
            U = arg < 0 ? init_u : snap_u[arg];
            D = arg < 0 ? init_d : snap_d[arg];
            cur = arg < 0 ? 0 : snap_step[arg];
        } else {   // FD_OP_ADJOINT: psi^k from psi^{k+1}, psi^{k+2}; gradient with u^k
            a.pcur = pcur;
            a.pprev = pprev;
            a.pnext = pprev;
            a.ufwd = U;
            a.with_grad = arg < nt;
            a.with_update = 1;
            if (!launch_adj(c, s, a, st)) return fail(FD_EUNSUPPORTED, "adjoint kernel not compiled");
            if (nrec > 0)
                launch_inject(pprev, s.rec, nrec, s.s->trace_adj + (size_t)(arg - 1) * nrec, s.v, c.ldv_y,
                              c.ldv_z, c.sp, s.nx, s.ny, s.nz, st);
            std::swap(pcur, pprev);
            R.launched(2);
        }
    }
    if (s.s->init_cur) {   // last gradient term f psi^1 (W u^0)
        a.pcur = pcur;
        a.pprev = pprev;
        a.pnext = pprev;
        a.ufwd = s.s->init_cur;
        a.with_grad = 1;
        a.with_update = 0;
        if (!launch_adj(c, s, a, st)) return fail(FD_EUNSUPPORTED, "adjoint kernel not compiled");
        R.launched();
    }
    if (c.g->check_finite && nrec > 0) {
        launch_check_finite(s.s->traces, (long long)nt * nrec, c.flags, st);
        R.launched();
    }
    return R.err;
}

// Every 2D shot advanced by one batched launch per step and stencil variant;
// variant groups run on parallel branches.
int enqueue_batched(const CallCtx& c, Recorder& R) {
    hipStream_t st = R.stream;
    const int nt = c.g->nt, ns = (int)c.shots.size();
    const BatchShot* dshots = (const BatchShot*)(c.ws + c.L.desc);
    const int2* jobs = (const int2*)(c.ws + c.L.jobs);
    long long maxn = 0;
    int maxrec = 0;
    for (const ShotCtx& s : c.shots) {
        maxn = std::max(maxn, s.npts);
        maxrec = std::max(maxrec, s.s->nrec);
        launch_rec_index(s.s->rec, s.s->nrec, 2, s.nx, 1, s.nz, s.rec, c.flags, st);
        R.launched();
    }
    // state: u^n in slot n&1, d in slot 2 (updated in place)
    launch_batch_copy(dshots, ns, maxn, 0, SLOT_INIT_CUR, st);
    launch_batch_copy(dshots, ns, maxn, 2, SLOT_INIT_DIFF, st);
    R.launched(2);
    // checkpoints into the callers' buffers (shots without one are skipped)
    const int K = c.K;
    if (K > 0) {
        launch_batch_copy(dshots, ns, maxn, SLOT_CKPT0, 2, st);
        launch_batch_copy(dshots, ns, maxn, SLOT_CKPT0 - 1, 0, st);
        R.launched(2);
    }
    BatchArgs a;
    a.shots = dshots;
    a.sp = c.sp;
    a.q = c.q;
    a.gather = 1;
    a.f_dcur = a.f_dnext = 2;
    R.fork(c.nbranch);
    bool ok = true;
    for (int n = 0; n < nt && ok; ++n) {
        a.step = n;
        a.f_ucur = n & 1;
        a.f_unext = (n + 1) & 1;
        for (const CallCtx::Group& g : c.groups) {
            a.jobs = jobs + g.job0;
            a.njobs = (int)g.njobs;
            ok = ok && launch_batch2d(a, g.shape, g.M, g.rows, R.on(g.branch));
        }
        R.launched((int)c.groups.size());
        if (K > 0 && (n + 1) % K == 0 && n + 1 < nt) {
            // pair j = (n+1)/K: (d^{n+1}, u^{n+1}) from slots 2 and (n+1)&1
            const int j = (n + 1) / K;
            for (const CallCtx::Group& g : c.groups) {
                launch_batch_copy(dshots + g.d0, g.dn, g.maxn, SLOT_CKPT0 - 2 * j, 2, R.on(g.branch));
                launch_batch_copy(dshots + g.d0, g.dn, g.maxn, SLOT_CKPT0 - 2 * j - 1, (n + 1) & 1, R.on(g.branch));
            }
            R.launched(2 * (int)c.groups.size());
        }
    }
    R.join();
    if (!ok) return fail(FD_EUNSUPPORTED, "batched kernel not compiled");
    const int last = nt & 1;
    launch_batch_gather(dshots, ns, maxrec, last, nt - 1, st);
    R.launched();
    for (const ShotCtx& s : c.shots) {
        if (s.s->final_diff) launch_copy(s.s->final_diff, s.bufA + 2 * s.npts, s.npts, st);
        if (s.s->final_cur) launch_copy(s.s->final_cur, s.bufA + last * s.npts, s.npts, st);
        if (c.g->check_finite && s.s->nrec > 0)
            launch_check_finite(s.s->traces, (long long)nt * s.s->nrec, c.flags, st);
        R.launched(3);
    }
    return R.err;
}

// Forward with checkpoints, then segment-wise recompute and adjoint, for
// every 2D shot at once (one launch per step and stencil variant, variant
// groups on parallel branches).  Each shot accumulates its gradient in its
// own arena field; the per-shot gradients are added into the model gradient
// at the end, shot after shot (deterministic).
int enqueue_batched_adjoint(const CallCtx& c, Recorder& R) {
    hipStream_t st = R.stream;
    const int nt = c.g->nt, K = c.K, ns = (int)c.shots.size();
    const int nseg = (nt + K - 1) / K;
    // saved checkpoints (every shot or none, checked in prepare): no forward pass
    const bool saved = c.shots[0].s->ckpt != nullptr;
    const AdjSlots S{nseg, K, saved};
    const BatchShot* dshots = (const BatchShot*)(c.ws + c.L.desc);
    const int2* jobs = (const int2*)(c.ws + c.L.jobs);
    long long maxn = 0;
    bool any_init = false;
    for (const ShotCtx& s : c.shots) {
        maxn = std::max(maxn, s.npts);
        any_init = any_init || s.s->init_cur;
        launch_rec_index(s.s->rec, s.s->nrec, 2, s.nx, 1, s.nz, s.rec, c.flags, st);
        R.launched();
    }
    auto copy_all = [&](int dst, int src) {
        launch_batch_copy(dshots, ns, maxn, dst, src, st);
        R.launched();
    };
    copy_all(SLOT_GACC, SLOT_ZERO);
    if (!saved) {
        copy_all(S.kU0, SLOT_INIT_CUR);
        copy_all(S.kD, SLOT_INIT_DIFF);
        copy_all(S.ck(0, 0), S.kD);
        copy_all(S.ck(0, 1), S.kU0);
    }
    // per-group helpers, each on the group's branch
    auto copy = [&](int dst, int src) {
        for (const CallCtx::Group& g : c.groups)
            launch_batch_copy(dshots + g.d0, g.dn, g.maxn, dst, src, R.on(g.branch));
        R.launched((int)c.groups.size());
    };
    bool ok = true;
    BatchArgs f;
    f.shots = dshots;
    f.sp = c.sp;
    f.q = c.q;
    auto fwd = [&]() {
        for (const CallCtx::Group& g : c.groups) {
            f.jobs = jobs + g.job0;
            f.njobs = (int)g.njobs;
            ok = ok && launch_batch2d(f, g.shape, g.M, g.rows, R.on(g.branch));
        }
        R.launched((int)c.groups.size());
    };
    BatchAdjArgs a;
    a.shots = dshots;
    a.gscale = grad_scale(c);
    a.gparam = c.gparam;
    a.sp = c.sp;
    auto adj = [&](bool inject, int k) {
        for (const CallCtx::Group& g : c.groups) {
            a.jobs = jobs + g.job0;
            a.njobs = (int)g.njobs;
            hipStream_t bs = R.on(g.branch);
            ok = ok && launch_batch_adj2d(a, g.shape, g.M, bs);
            if (inject) launch_batch_inject(dshots + g.d0, g.dn, g.maxrec, a.f_pprev, k, c.sp, bs);
        }
        R.launched((int)c.groups.size() * (inject ? 2 : 1));
    };

    R.fork(c.nbranch);
    const int tail = ((nt - 1) / K) * K;
    int cur = S.kU0, last = S.kU0;
    for (int n = 0; n < nt && ok && !saved; ++n) {
        f.step = n;
        f.gather = 1;
        f.f_dcur = f.f_dnext = S.kD;
        if (n < tail) {
            f.f_ucur = cur;
            f.f_unext = cur ^ 1;
        } else {
            const int i = n - tail;
            f.f_ucur = i == 0 ? cur : S.seg(i - 1);
            f.f_unext = S.seg(i);
        }
        fwd();
        last = f.f_unext;
        if (n < tail) {
            cur ^= 1;
            if ((n + 1) % K == 0 && n + 1 < nt) {
                copy(S.ck((n + 1) / K, 0), S.kD);
                copy(S.ck((n + 1) / K, 1), cur);
            }
        }
    }
    if (!saved) {
        for (const CallCtx::Group& g : c.groups)
            launch_batch_gather(dshots + g.d0, g.dn, g.maxrec, last, nt - 1, R.on(g.branch));
        R.launched((int)c.groups.size());
    }
    R.cut();
    copy(S.psiA(), SLOT_ZERO);
    copy(S.psiB(), SLOT_ZERO);
    int pcur = S.psiA(), pprev = S.psiB();
    f.gather = 0;
    for (int j = nseg - 1; j >= 0 && ok; --j) {
        const int s0 = j * K, e0 = std::min(nt, s0 + K);
        for (int step = s0; step < e0 && (j < nseg - 1 || saved); ++step) {
            const int i = step - s0;
            f.step = step;
            f.f_ucur = i == 0 ? S.ck(j, 1) : S.seg(i - 1);
            f.f_dcur = i == 0 ? S.ck(j, 0) : S.dseg();
            f.f_dnext = S.dseg();
            f.f_unext = S.seg(i);
            fwd();
        }
        for (int k = e0; k > s0; --k) {
            a.f_pcur = pcur;
            a.f_pprev = a.f_pnext = pprev;
            a.f_ufwd = S.seg(k - s0 - 1);
            a.with_grad = k < nt;
            a.with_update = 1;
            adj(true, k);
            std::swap(pcur, pprev);
        }
        R.cut();
    }
    if (any_init) {
        a.f_pcur = pcur;
        a.f_pprev = pprev;
        a.f_pnext = -1;
        a.f_ufwd = SLOT_INIT_CUR;
        a.with_grad = 1;
        a.with_update = 0;
        adj(false, 0);
    }
    R.join();
    if (!ok) return fail(FD_EUNSUPPORTED, "batched kernel not compiled");
    for (const ShotCtx& s : c.shots) {
        launch_accum2d(c.grad + model_offset(c, *s.s), c.ldv_y, s.bufA + (long long)S.gacc() * s.npts,
                       s.nx, s.nz, st);
        if (c.g->check_finite && s.s->nrec > 0 && !saved)
            launch_check_finite(s.s->traces, (long long)nt * s.s->nrec, c.flags, st);
        R.launched(2);
    }
    return R.err;
}

// Relative cost of one update with stencil (shape, M): stencil points plus
// a fixed part for the loads, the update and the store.  A launch adds a
// fixed cost of its own (ramp-up and drain, about 4.3 us on gfx950, where a
// 10^6-point window costs about 0.021 us per stencil point): kLaunchCost in
// the same units (points x update_cost).  Without it a group of short,
// latency-bound launches looks cheap and the balancing stacks several of
// them on one branch, where their latencies add up every step.
constexpr double kLaunchCost = 2.0e8;

double update_cost(int shape, int M) {
    const int P = shape == SH_CROSS ? 4 * M + 1 : (shape == SH_RHOMBUS ? 2 * M * M + 2 * M + 1
                                                                       : (2 * M + 1) * (2 * M + 1));
    return P + 24.0;
}

// Descriptors and work list of a batched call, built on the host: shots
// sorted by stencil variant, one contiguous descriptor and job range per
// variant, groups spread over the branches by decreasing cost (each to the
// least loaded branch).
void build_batch_blob(CallCtx& c, int mode) {
    const int nshots = (int)c.shots.size();
    std::vector<int> order(nshots);
    for (int i = 0; i < nshots; ++i) order[i] = i;
    auto variant = [&](int i) { return c.shots[i].st.shape * 8 + c.shots[i].st.M - 1; };
    std::stable_sort(order.begin(), order.end(), [&](int x, int y) { return variant(x) < variant(y); });
    std::vector<BatchShot> desc(nshots);
    std::vector<int2> jobs;
    jobs.reserve((size_t)c.L.njobs);
    const AdjSlots S{mode == MODE_ADJ_SEGMENT ? (c.g->nt + c.K - 1) / c.K : 0, c.K,
                     mode == MODE_ADJ_SEGMENT && c.shots[0].s->ckpt != nullptr};
    c.groups.clear();
    std::vector<double> gcost;
    for (int k = 0; k < nshots; ++k) {
        const ShotCtx& s = c.shots[order[k]];
        if (c.groups.empty() || variant(order[k]) != variant(order[k - 1])) {
            CallCtx::Group g;
            g.shape = s.st.shape;
            g.M = s.st.M;
            // forward steps: the stencil's batched tile (fd_set_batch_tile;
            // by default 64 x 32 for dense shapes, 64 x 16 for crosses: with
            // the groups running concurrently the dense groups' taller tiles
            // win, 8-stencil 1001^2 step 64.8 -> 60.4 ms); the adjoint's job
            // list (shared with its recompute) stays at 4 rows
            g.rows = mode == MODE_FORWARD ? batch_forward_rows(s.st) : batch_rows();
            g.d0 = k;
            g.dn = 0;
            g.job0 = (long long)jobs.size();
            g.njobs = 0;
            g.maxn = 0;
            g.maxrec = 0;
            g.branch = 0;
            c.groups.push_back(g);
            gcost.push_back(kLaunchCost);
        }
        CallCtx::Group& g = c.groups.back();
        BatchShot& d = desc[k];
        std::memset(&d, 0, sizeof d);
        d.arena = s.bufA;
        d.npts = s.npts;
        d.v = s.v;
        d.ldv = c.ldv_y;
        d.nx = s.nx;
        d.nz = s.nz;
        d.ntiles = shot_tiles2d(*s.s, g.rows, &d.tiles_x);
        d.src = s.src;
        d.wavelet = s.s->wavelet;
        d.nrec = s.s->nrec;
        d.rec_lin = s.rec;
        d.traces = s.s->traces;
        d.trace_adj = s.s->trace_adj;
        d.init_diff = s.s->init_diff;
        d.init_cur = s.s->init_cur;
        d.gacc = mode == MODE_ADJ_SEGMENT ? s.bufA + (long long)S.gacc() * s.npts : nullptr;
        d.ckpt = s.s->ckpt;
        d.variant = variant(order[k]);
        d.w = s.st.w32;
        for (int t = 0; t < d.ntiles; ++t) jobs.push_back(make_int2(k, t));
        g.dn++;
        g.njobs += d.ntiles;
        g.maxn = std::max(g.maxn, s.npts);
        g.maxrec = std::max(g.maxrec, s.s->nrec);
        gcost.back() += (double)s.npts * update_cost(s.st.shape, s.st.M);
    }
    const int ng = (int)c.groups.size();
    c.nbranch = std::min(ng, kBranches);
    std::vector<int> by_cost(ng);
    for (int i = 0; i < ng; ++i) by_cost[i] = i;
    std::stable_sort(by_cost.begin(), by_cost.end(), [&](int x, int y) { return gcost[x] > gcost[y]; });
    std::vector<double> load(c.nbranch, 0.0);
    for (int gi : by_cost) {
        const int b = (int)(std::min_element(load.begin(), load.end()) - load.begin());
        c.groups[gi].branch = b;
        load[b] += gcost[gi];
    }
    c.blob_off = c.L.desc;
    const size_t jobs_rel = c.L.jobs - c.L.desc;
    c.blob.assign(jobs_rel + sizeof(int2) * jobs.size(), 0);
    std::memcpy(c.blob.data(), desc.data(), sizeof(BatchShot) * desc.size());
    std::memcpy(c.blob.data() + jobs_rel, jobs.data(), sizeof(int2) * jobs.size());
}

int enqueue_call(const CallCtx& c, int mode, Recorder& R) {
    std::lock_guard<std::mutex> lk(g_branch_mu);   // the branches' events are shared
    int rc = FD_OK;
    launch_fill_i32(c.flags, FLAG_COUNT, 0, R.stream);
    const long long mpts = c.g->n[0] * (c.g->ndim == 3 ? c.g->n[1] : 1) * c.g->n[2];
    launch_vprep(c.vel, c.vfield, mpts, c.g->dt / c.g->h, c.c_lim, c.flags, R.stream);
    R.launched(2);
    if (use_batch(c.g, (int)c.shots.size(), mode))
        return mode == MODE_FORWARD ? enqueue_batched(c, R) : enqueue_batched_adjoint(c, R);
    // forward shots own their fields: unless FD_NO_BATCH asks for shot after
    // shot, they run on parallel branches (adjoint shots share the checkpoint
    // and adjoint fields and the gradient, so they stay in sequence)
    const int ns = (int)c.shots.size();
    const bool par = mode == MODE_FORWARD && ns > 1 && !(c.g->flags & FD_NO_BATCH);
    if (par) R.fork(ns);
    for (int i = 0; i < ns; ++i) {
        if (par) R.active = i;
        rc = mode == MODE_FORWARD ? enqueue_forward_shot(c, c.shots[i], c.K > 0 ? c.shots[i].s->ckpt : nullptr,
                                                         c.K, nullptr, R)
           : mode == MODE_ADJ_SEGMENT ? enqueue_adjoint_shot(c, c.shots[i], R)
                                      : enqueue_adjoint_revolve(c, c.shots[i], R);
        if (rc) break;
    }
    R.active = -1;
    R.join();
    return rc ? rc : R.err;
}

int get_capture_stream(int dev, hipStream_t* out) {
    auto it = g_graphs.capture_streams.find(dev);
    if (it != g_graphs.capture_streams.end()) {
        *out = it->second;
        return FD_OK;
    }
    hipStream_t s;
    HIP_OK(hipStreamCreateWithFlags(&s, hipStreamNonBlocking));
    g_graphs.capture_streams[dev] = s;
    *out = s;
    return FD_OK;
}

int run_direct(CallCtx& c, int mode, hipStream_t user) {
    if (!c.blob.empty()) {
        HIP_OK(hipMemcpyAsync(c.ws + c.blob_off, c.blob.data(), c.blob.size(), hipMemcpyHostToDevice, user));
        HIP_OK(hipStreamSynchronize(user));   // the host copy of the blob is freed on return
    }
    Recorder R;
    R.stream = user;
    int rc = get_branches(&R.br);
    if (rc) return rc;
    rc = enqueue_call(c, mode, R);
    if (rc) return rc;
    HIP_OK(hipGetLastError());
    return FD_OK;
}

// ---------------------------------------------------------------------------
// fixed device scratch for fd_forward_noalloc: one array per GPU, resident
// until the process ends.  Host code never passes `scratch` itself to a
// kernel (on the host it only names the symbol); kernels get the device
// address that hipGetSymbolAddress returns for the current device, taken
// once per device at that device's first call.
// ---------------------------------------------------------------------------
__device__ __align__(256) unsigned char scratch[FD_NOALLOC_SCRATCH_BYTES];
std::mutex g_scratch_mu;
std::map<int, void*> g_scratch_ptr;

int scratch_address(void** out) {
    int dev = 0;
    HIP_OK(hipGetDevice(&dev));
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    auto it = g_scratch_ptr.find(dev);
    if (it == g_scratch_ptr.end()) {
        void* ptr = nullptr;
        HIP_OK(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
        if (!ptr) return fail(FD_EDEVICE, "hipGetSymbolAddress returned no address for the scratch array");
        it = g_scratch_ptr.emplace(dev, ptr).first;
    }
    *out = it->second;
    return FD_OK;
}

// Direct launches on the caller's stream with no library-owned streams,
// events, graphs or pinned buffers (a single shot needs no branches).
int run_direct_noalloc(CallCtx& c, hipStream_t user) {
    Recorder R;
    R.stream = user;
    R.br = nullptr;
    const int rc = enqueue_call(c, MODE_FORWARD, R);
    if (rc) return rc;
    HIP_OK(hipGetLastError());
    return FD_OK;
}

int run_call(CallCtx& c, int mode, hipStream_t user) {
    if (c.g->flags & FD_NO_GRAPH) return run_direct(c, mode, user);
    int dev = 0;
    HIP_OK(hipGetDevice(&dev));
    std::vector<uint64_t> key;
    key.push_back((uint64_t)dev);
    key.push_back((uint64_t)mode);
    key.push_back((uint64_t)c.K);
    key.push_back((uint64_t)c.gparam);
    key.push_back((uint64_t)(uintptr_t)c.grad);
    key_push(key, c.g, sizeof(fd_grid));
    key.push_back((uint64_t)(uintptr_t)c.vel);
    key.push_back((uint64_t)(uintptr_t)c.ws);
    for (const ShotCtx& s : c.shots) {
        key_push(key, s.s, sizeof(fd_shot));
        key.push_back(((uint64_t)s.st.rows << 32) | (uint32_t)s.st.zchunk);
        key.push_back(((uint64_t)s.st.tsteps << 32) | (uint32_t)s.st.brows);
    }
    std::lock_guard<std::mutex> lk(g_graphs.mu);
    GraphCache::Entry* entry = nullptr;
    for (auto it = g_graphs.lru.begin(); it != g_graphs.lru.end(); ++it) {
        if (it->key == key) {
            g_graphs.lru.splice(g_graphs.lru.begin(), g_graphs.lru, it);
            entry = &g_graphs.lru.front();
            break;
        }
    }
    if (!entry) {
        hipStream_t cs;
        int rc = get_capture_stream(dev, &cs);
        if (rc) return rc;
        Recorder R;
        R.stream = cs;
        R.capturing = true;
        rc = get_branches(&R.br);
        if (rc) return rc;
        HIP_OK(hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal));
        rc = enqueue_call(c, mode, R);
        if (R.capturing) {
            hipGraph_t graph = nullptr;
            hipError_t e = hipStreamEndCapture(cs, &graph);
            hipGraphExec_t exec = nullptr;
            if (e == hipSuccess && !rc && !R.err && R.nodes > 0)
                e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
            if (graph) hipGraphDestroy(graph);
            if (exec) R.execs.push_back(exec);
            if (e != hipSuccess && !rc && !R.err)
                R.err = fail(FD_EDEVICE, "graph capture failed: %s", hipGetErrorString(e));
        }
        if (rc || R.err) {
            for (hipGraphExec_t x : R.execs) hipGraphExecDestroy(x);
            if (rc) return rc;
            // capture is an optimisation: queue the same work directly
            (void)hipGetLastError();
            g_graph_fallbacks++;
            return run_direct(c, mode, user);
        }
        GraphCache::Entry ne;
        ne.key = key;
        ne.execs = R.execs;
        if (!c.blob.empty()) {
            HIP_OK(hipHostMalloc(&ne.pinned, c.blob.size(), hipHostMallocDefault));
            std::memcpy(ne.pinned, c.blob.data(), c.blob.size());
            ne.pinned_bytes = c.blob.size();
        }
        g_graphs.lru.push_front(ne);
        entry = &g_graphs.lru.front();
        while (g_graphs.lru.size() > GraphCache::kCap) {
            GraphCache::Entry& old = g_graphs.lru.back();
            for (hipGraphExec_t x : old.execs) hipGraphExecDestroy(x);
            if (old.pinned) {
                (void)hipDeviceSynchronize();   // its last upload may still be in flight
                (void)hipHostFree(old.pinned);
            }
            g_graphs.lru.pop_back();
        }
    }
    if (entry->pinned)
        HIP_OK(hipMemcpyAsync(c.ws + c.blob_off, entry->pinned, entry->pinned_bytes, hipMemcpyHostToDevice, user));
    for (hipGraphExec_t x : entry->execs) HIP_OK(hipGraphLaunch(x, user));
    return FD_OK;
}

int finish_checks(const CallCtx& c, hipStream_t user) {
    if (!c.g->check_finite) return FD_OK;
    HIP_OK(hipStreamSynchronize(user));
    int flags[FLAG_COUNT];
    HIP_OK(hipMemcpy(flags, c.flags, sizeof flags, hipMemcpyDeviceToHost));
    if (flags[FLAG_BAD_VEL]) return fail(FD_EINVAL, "%d velocities are not positive and finite", flags[FLAG_BAD_VEL]);
    if (flags[FLAG_UNSTABLE_VEL])
        return fail(FD_EUNSTABLE, "%d velocities c have c dt / h above the stability limit %.6g of the call's stencils",
                    flags[FLAG_UNSTABLE_VEL], c.c_lim);
    if (flags[FLAG_BAD_REC]) return fail(FD_EINVAL, "%d receiver coordinates lie outside their window", flags[FLAG_BAD_REC]);
    if (flags[FLAG_NONFINITE]) return fail(FD_ENONFINITE, "%d trace samples are not finite", flags[FLAG_NONFINITE]);
    return FD_OK;
}

int prepare(CallCtx& c, const fd_grid* g, const float* vel, const fd_shot* shots, int nshots, int mode,
            int K, void* workspace, size_t ws_bytes) {
    int rc = check_grid(g);
    if (rc) return rc;
    if (!vel) return fail(FD_EINVAL, "vel is NULL");
    if (!shots || nshots < 1) return fail(FD_EINVAL, "need at least one shot");
    if (mode == MODE_ADJ_SEGMENT && (K < 1 || K > g->nt)) return fail(FD_EINVAL, "ckpt_every must be in [1, nt]");
    if (mode == MODE_FORWARD && (K < 0 || K > g->nt)) return fail(FD_EINVAL, "ckpt_every must be in [0, nt]");
    const int nsaved = saved_count(shots, nshots);
    if (nsaved > 0 && mode == MODE_FORWARD && K == 0)
        return fail(FD_EINVAL, "shots pass checkpoint buffers but ckpt_every is 0");
    if (nsaved > 0 && mode == MODE_ADJ_REVOLVE)
        return fail(FD_EINVAL, "saved checkpoints (fd_shot.ckpt) need segment checkpointing");
    if (nsaved > 0 && nsaved < nshots && mode == MODE_ADJ_SEGMENT && use_batch(g, nshots, mode))
        return fail(FD_EINVAL, "a batched adjoint needs saved checkpoints for every shot or for none");
    if (mode == MODE_ADJ_REVOLVE && (K < 0 || K > g->nt)) return fail(FD_EINVAL, "nsnap must be in [0, nt]");
    c.g = g;
    c.vel = vel;
    c.nshots = nshots;
    c.K = K;
    c.L = make_layout(g, shots, nshots, mode, K);
    if (!workspace) return fail(FD_EINVAL, "workspace is NULL");
    if ((uintptr_t)workspace % 256) return fail(FD_EINVAL, "workspace must be 256-byte aligned");
    if (ws_bytes < c.L.total)
        return fail(FD_ENOMEM, "workspace too small: %zu < %zu bytes", ws_bytes, c.L.total);
    c.ws = (char*)workspace;
    c.flags = (int*)(c.ws + c.L.flags);
    c.vfield = (float*)(c.ws + c.L.v);
    // model strides: row (y) and plane (z); in 2D the z stride is the row
    // length, and the 2D kernels address rows with ldv_y (== ldv_z)
    c.ldv_y = g->n[0];
    c.ldv_z = g->n[0] * (g->ndim == 3 ? g->n[1] : 1);
    c.sp.nb = g->nb;
    c.sp.escale = (float)(0.5 * g->eta_max * g->dt);
    c.sp.inv_nb = g->nb > 0 ? (float)(1.0 / g->nb) : 0.f;
    c.q = (float)(g->dt * g->dt / std::pow(g->h, g->ndim));
    c.grad = nullptr;
    c.c_lim = HUGE_VAL;
    for (int i = 0; i < nshots; ++i) {
        ShotCtx s;
        rc = check_shot(g, shots[i], i, mode != MODE_FORWARD, &s.st);
        if (rc) return rc;
        c.c_lim = std::min(c.c_lim, s.st.cfl);
        s.s = &shots[i];
        s.nx = (int)shots[i].extent[0];
        s.ny = g->ndim == 3 ? (int)shots[i].extent[1] : 1;
        s.nz = (int)shots[i].extent[2];
        s.npts = window_points(shots[i], g->ndim);
        s.v = c.vfield + model_offset(c, shots[i]);
        s.bufA = (float*)(c.ws + c.L.shots[i].arena);
        s.bufB = s.bufA + s.npts;
        s.rec = (long long*)(c.ws + c.L.shots[i].rec);
        const int* p = shots[i].src;
        s.src = g->ndim == 2 ? (long long)p[2] * s.nx + p[0]
                             : ((long long)p[2] * s.ny + p[1]) * s.nx + p[0];
        c.shots.push_back(s);
    }
    if (use_batch(g, nshots, mode)) build_batch_blob(c, mode);
    return FD_OK;
}

// ---------------------------------------------------------------------------
// dispersion metrics (Appendix A): rocFFT plans and receiver chunking
// ---------------------------------------------------------------------------
// Plans are cached per (device, kind, length, batch) with their work buffer
// and execution info; like the graph cache they live until the process ends.
struct FftPlan {
    int dev, kind;            // kind 0: real forward, 1: complex inverse (in place)
    size_t len, batch;
    rocfft_plan plan = nullptr;
    rocfft_execution_info info = nullptr;
    void* work = nullptr;
    size_t work_bytes = 0;
};
std::list<FftPlan> g_fft;   // stable addresses for the returned plans
std::mutex g_fft_mu;

int fft_plan(int kind, size_t len, size_t batch, FftPlan** out) {
    std::lock_guard<std::mutex> lk(g_fft_mu);
    int dev = 0;
    HIP_OK(hipGetDevice(&dev));
    for (FftPlan& p : g_fft)
        if (p.dev == dev && p.kind == kind && p.len == len && p.batch == batch) {
            *out = &p;
            return FD_OK;
        }
    static bool setup = false;
    if (!setup) {
        if (rocfft_setup() != rocfft_status_success) return fail(FD_EDEVICE, "rocfft_setup failed");
        setup = true;
    }
    FftPlan p;
    p.dev = dev;
    p.kind = kind;
    p.len = len;
    p.batch = batch;
    const rocfft_status st = rocfft_plan_create(
        &p.plan, kind == 0 ? rocfft_placement_notinplace : rocfft_placement_inplace,
        kind == 0 ? rocfft_transform_type_real_forward : rocfft_transform_type_complex_inverse,
        rocfft_precision_double, 1, &len, batch, nullptr);
    if (st != rocfft_status_success) return fail(FD_EDEVICE, "rocfft_plan_create failed (%d)", (int)st);
    if (rocfft_plan_get_work_buffer_size(p.plan, &p.work_bytes) != rocfft_status_success)
        return fail(FD_EDEVICE, "rocfft_plan_get_work_buffer_size failed");
    if (rocfft_execution_info_create(&p.info) != rocfft_status_success)
        return fail(FD_EDEVICE, "rocfft_execution_info_create failed");
    if (p.work_bytes) {
        HIP_OK(hipMalloc(&p.work, p.work_bytes));
        if (rocfft_execution_info_set_work_buffer(p.info, p.work, p.work_bytes) != rocfft_status_success)
            return fail(FD_EDEVICE, "rocfft_execution_info_set_work_buffer failed");
    }
    g_fft.push_back(p);
    *out = &g_fft.back();
    return FD_OK;
}

int fft_run(FftPlan* p, void* in, void* out, hipStream_t st) {
    std::lock_guard<std::mutex> lk(g_fft_mu);
    if (rocfft_execution_info_set_stream(p->info, st) != rocfft_status_success)
        return fail(FD_EDEVICE, "rocfft_execution_info_set_stream failed");
    void* ib[1] = {in};
    void* ob[1] = {out};
    if (rocfft_execute(p->plan, ib, out ? ob : nullptr, p->info) != rocfft_status_success)
        return fail(FD_EDEVICE, "rocfft_execute failed");
    return FD_OK;
}

// receivers per chunk: at most 64, and the two CWT fields of a chunk within
// 512 MiB
int disp_chunk(int nt, int nrec, int nscale) {
    long long r = std::min(nrec, 64);
    if (nscale > 0) {
        const long long per = 2LL * nscale * nt * 16;
        r = std::min(r, std::max(1LL, (512LL << 20) / per));
    }
    return (int)r;
}

struct DispLayout {
    size_t xa, xb, fa, fb, wa, wb, total;
};

DispLayout disp_layout(int nt, int nrec, int nscale) {
    const int R = disp_chunk(nt, nrec, nscale);
    const size_t nh = (size_t)nt / 2 + 1;
    DispLayout L;
    size_t off = 0;
    L.xa = off; off = align256(off + 8 * (size_t)R * nt);
    L.xb = off; off = align256(off + 8 * (size_t)R * nt);
    L.fa = off; off = align256(off + 16 * (size_t)R * nh);
    L.fb = off; off = align256(off + 16 * (size_t)R * nh);
    L.wa = L.wb = 0;
    if (nscale > 0) {
        L.wa = off; off = align256(off + 16 * (size_t)R * nscale * nt);
        L.wb = off; off = align256(off + 16 * (size_t)R * nscale * nt);
    }
    L.total = off;
    return L;
}

}  // namespace

// ---------------------------------------------------------------------------
// C ABI
// ---------------------------------------------------------------------------
extern "C" {

const char* fd_last_error(void) { return g_err.c_str(); }

int fd_orbits_n(int ndim, int shape, int M, int N, int* reps, int* counts, int* nw) {
    if (!nw) return fail(FD_EINVAL, "nw is NULL");
    if (!valid_shape(ndim, shape, M, N))
        return fail(FD_EINVAL, "invalid ndim/shape/M/N (%d, %d, %d, %d)", ndim, shape, M, N);
    std::vector<Orbit> o = make_orbits(ndim, shape, M, N);
    *nw = (int)o.size();
    for (size_t i = 0; i < o.size(); ++i) {
        if (reps)
            for (int a = 0; a < ndim; ++a) reps[i * ndim + a] = o[i].rep[a];
        if (counts) counts[i] = o[i].count;
    }
    return FD_OK;
}

int fd_orbits(int ndim, int shape, int M, int* reps, int* counts, int* nw) {
    return fd_orbits_n(ndim, shape, M, 0, reps, counts, nw);
}

int fd_weights_set_n(int ndim, int shape, int M, int N, const double* w, int nw, int* stencil_id) {
    if (!stencil_id || !w) return fail(FD_EINVAL, "NULL argument");
    if (!valid_shape(ndim, shape, M, N))
        return fail(FD_EINVAL, "invalid ndim/shape/M/N (%d, %d, %d, %d)", ndim, shape, M, N);
    std::vector<Orbit> o = make_orbits(ndim, shape, M, N);
    if (nw != (int)o.size()) return fail(FD_EINVAL, "expected %zu weights, got %d", o.size(), nw);
    if ((int)o.size() > kMaxOrbits) return fail(FD_EUNSUPPORTED, "too many orbits (%zu)", o.size());
    double sum = 0.0, asum = 0.0;
    for (int i = 0; i < nw; ++i) {
        if (!std::isfinite(w[i])) return fail(FD_EINVAL, "weight %d is not finite", i);
        sum += o[i].count * w[i];
        asum += o[i].count * std::fabs(w[i]);
    }
    if (!(asum > 0)) return fail(FD_EINVAL, "all weights are zero");
    if (std::fabs(sum) > 1e-9 * asum)
        return fail(FD_EINVAL, "weights violate the zero-sum condition: sum count*w = %.3g", sum);
    Symbol S = make_symbol(ndim, shape, M, N, o, w);
    double mneg, mpos;
    symbol_extrema(S, &mneg, &mpos);
    if (mpos > 1e-9 * asum) return fail(FD_EUNSTABLE, "stencil symbol is positive (%.3g): unstable for every dt", mpos);
    if (!(mneg > 0)) return fail(FD_EINVAL, "stencil symbol is identically zero");
    const int ks = kernel_shape(shape, M, N);
    Stencil st;
    st.ndim = ndim;
    st.shape = ks;
    st.ushape = shape;
    st.N = N;
    st.M = M;
    st.nw = nw;
    st.w64.assign(w, w + nw);
    std::memset(&st.w32, 0, sizeof st.w32);
    if (ks == SH_CROSS) {
        // cross kernels index weights by cross orbit (the axis offsets 0..M)
        for (int i = 0; i < nw; ++i)
            if (o[i].rep[1] == 0 && o[i].rep[2] == 0) st.w32.w[o[i].rep[0]] = (float)w[i];
    } else {
        for (int i = 0; i < nw; ++i) st.w32.w[i] = (float)w[i];
    }
    if (ndim == 2) {
        for (int dx = 0; dx <= M; ++dx)
            for (int dz = 0; dz <= M; ++dz) {
                int a = std::max(dx, dz), b = std::min(dx, dz);
                for (int i = 0; i < nw; ++i)
                    if (o[i].rep[0] == a && o[i].rep[1] == b) st.w32.wd[dx * (M + 1) + dz] = (float)w[i];
            }
        for (int dz = 1; dz <= M; ++dz) {
            double acc = st.w32.wd[dz];
            for (int dx = 1; dx <= M; ++dx) acc += 2.0 * (double)st.w32.wd[dx * (M + 1) + dz];
            st.w32.wc[dz] = (float)acc;
        }
        // z extent of the offset group of each column dx >= 1 (the set of dz
        // with (dx, dz) in the shape is 0..mz for every shape here)
        for (int dx = 1; dx <= M; ++dx) {
            int mz = 0;
            for (int dz = 1; dz <= M; ++dz) {
                const int a = std::max(dx, dz), b = std::min(dx, dz);
                if (in_shape(2, shape, M, N, a, b, 0)) mz = dz;
            }
            st.w32.mz[dx] = mz;
        }
    }
    if (ndim == 3 && ks == SH_RHOMBUS) {
        // the 3D L1-ball kernel folds the in-plane groups' centre terms into
        // the z differences of the centre column:
        // wc[dz] = w(0,0,dz) + sum_{a >= b >= 0, 1 <= a+b <= M-dz} n_ab w(a,b,dz)
        auto wof = [&](int x, int y, int z) -> double {
            int t[3] = {x, y, z};
            std::sort(t, t + 3, [](int p, int q) { return p > q; });
            for (int i = 0; i < nw; ++i)
                if (o[i].rep[0] == t[0] && o[i].rep[1] == t[1] && o[i].rep[2] == t[2]) return (double)(float)w[i];
            return 0.0;
        };
        for (int dz = 1; dz <= M; ++dz) {
            double acc = wof(0, 0, dz);
            for (int s = 1; s <= M - dz; ++s)
                for (int b = 0; b <= s / 2; ++b) {
                    const int a = s - b;
                    acc += ((b == 0 || a == b) ? 4.0 : 8.0) * wof(a, b, dz);
                }
            st.w32.wc[dz] = (float)acc;
        }
    }
    st.cfl = 2.0 / std::sqrt(mneg);
    st.rows = default_rows(ndim, ks, M);
    st.zchunk = ndim == 3 ? 512 : 64;
    st.tsteps = 1;
    st.brows = 0;
    std::lock_guard<std::mutex> lk(g_mu);
    for (size_t i = 0; i < g_stencils.size(); ++i) {
        const Stencil& e = g_stencils[i];
        if (e.ndim == ndim && e.ushape == shape && e.N == N && e.M == M && e.w64 == st.w64) {
            *stencil_id = (int)i;
            return FD_OK;
        }
    }
    if ((int)g_stencils.size() >= FD_MAX_STENCILS) return fail(FD_EUNSUPPORTED, "too many stencils registered");
    g_stencils.push_back(st);
    *stencil_id = (int)g_stencils.size() - 1;
    return FD_OK;
}

int fd_weights_set(int ndim, int shape, int M, const double* w, int nw, int* stencil_id) {
    return fd_weights_set_n(ndim, shape, M, 0, w, nw, stencil_id);
}

int fd_cfl_limit(int stencil_id, double* c_lim) {
    Stencil st;
    if (!c_lim) return fail(FD_EINVAL, "c_lim is NULL");
    if (!get_stencil(stencil_id, &st)) return fail(FD_EINVAL, "unknown stencil id %d", stencil_id);
    *c_lim = st.cfl;
    return FD_OK;
}

int fd_set_tile(int stencil_id, int rows, int zchunk) {
    std::lock_guard<std::mutex> lk(g_mu);
    if (stencil_id < 0 || stencil_id >= (int)g_stencils.size()) return fail(FD_EINVAL, "unknown stencil id");
    if (rows != 1 && rows != 2 && rows != 4 && rows != 8) return fail(FD_EINVAL, "rows must be 1, 2, 4 or 8");
    if (zchunk < 8 || zchunk > 4096 || zchunk % 8) return fail(FD_EINVAL, "zchunk must be a multiple of 8 in [8, 4096]");
    Stencil& s = g_stencils[stencil_id];
    const bool have = s.ndim == 2 ? have_fwd2d(s.shape, s.M, rows) : have_fwd3d(s.shape, s.M, rows);
    if (!have) return fail(FD_EUNSUPPORTED, "no kernel compiled for rows = %d", rows);
    s.rows = rows;
    s.zchunk = zchunk;
    return FD_OK;
}

int fd_set_time_block(int stencil_id, int steps) {
    std::lock_guard<std::mutex> lk(g_mu);
    if (stencil_id < 0 || stencil_id >= (int)g_stencils.size()) return fail(FD_EINVAL, "unknown stencil id");
    if (steps != 1 && steps != 2) return fail(FD_EINVAL, "steps must be 1 or 2");
    if (steps == 2) return fail(FD_EUNSUPPORTED, "two time steps per launch are not compiled");
    g_stencils[stencil_id].tsteps = 1;
    return FD_OK;
}

int fd_get_time_block(int stencil_id, int* steps) {
    Stencil st;
    if (!steps) return fail(FD_EINVAL, "steps is NULL");
    if (!get_stencil(stencil_id, &st)) return fail(FD_EINVAL, "unknown stencil id");
    *steps = st.tsteps;
    return FD_OK;
}

int fd_get_tile(int stencil_id, int* rows, int* zchunk) {
    Stencil st;
    if (!get_stencil(stencil_id, &st)) return fail(FD_EINVAL, "unknown stencil id");
    if (rows) *rows = st.rows;
    if (zchunk) *zchunk = st.zchunk;
    return FD_OK;
}

int fd_set_batch_tile(int stencil_id, int rows) {
    std::lock_guard<std::mutex> lk(g_mu);
    if (stencil_id < 0 || stencil_id >= (int)g_stencils.size()) return fail(FD_EINVAL, "unknown stencil id");
    if (rows != 0 && rows != 4 && rows != 8) return fail(FD_EINVAL, "batched rows must be 0, 4 or 8");
    Stencil& s = g_stencils[stencil_id];
    if (s.ndim != 2) return fail(FD_EUNSUPPORTED, "batched calls are 2D only");
    if (rows == 8 && s.shape == SH_CROSS) return fail(FD_EUNSUPPORTED, "no batched cross kernel for rows = 8");
    s.brows = rows;
    return FD_OK;
}

int fd_get_batch_tile(int stencil_id, int* rows) {
    Stencil st;
    if (!get_stencil(stencil_id, &st)) return fail(FD_EINVAL, "unknown stencil id");
    if (st.ndim != 2) return fail(FD_EUNSUPPORTED, "batched calls are 2D only");
    if (rows) *rows = batch_forward_rows(st);
    return FD_OK;
}

size_t fd_workspace_bytes(const fd_grid* g, const fd_shot* shots, int nshots, int mode, int ckpt_every) {
    if (check_grid(g) || !shots || nshots < 1 || mode < 0 || mode > 1) return 0;
    if (mode == 1 && (ckpt_every < 1 || ckpt_every > g->nt)) return 0;
    return make_layout(g, shots, nshots, mode, mode == 1 ? ckpt_every : 1).total;
}

int fd_forward(const fd_grid* g, const float* vel, const fd_shot* shots, int nshots, int ckpt_every,
               void* workspace, size_t ws_bytes, void* hip_stream) {
    g_err.clear();
    CallCtx c;
    int rc = prepare(c, g, vel, shots, nshots, 0, ckpt_every, workspace, ws_bytes);
    if (rc) return rc;
    hipStream_t st = (hipStream_t)hip_stream;
    rc = run_call(c, 0, st);
    if (rc) return rc;
    return finish_checks(c, st);
}

int fd_forward_noalloc(const fd_grid* g, const float* vel, const fd_shot* shot, void* hip_stream) {
    g_err.clear();
    if (!shot) return fail(FD_EINVAL, "shot is NULL");
    if (check_grid(g)) return FD_EINVAL;
    const size_t need = make_layout(g, shot, 1, MODE_FORWARD, 0).total;
    if (need > FD_NOALLOC_SCRATCH_BYTES)
        return fail(FD_ENOMEM, "fd_forward_noalloc: this call needs %zu bytes of scratch, the fixed array holds %zu "
                    "(use fd_forward with a workspace)", need, (size_t)FD_NOALLOC_SCRATCH_BYTES);
    void* ws = nullptr;
    int rc = scratch_address(&ws);
    if (rc) return rc;
    CallCtx c;
    rc = prepare(c, g, vel, shot, 1, MODE_FORWARD, 0, ws, FD_NOALLOC_SCRATCH_BYTES);
    if (rc) return rc;
    hipStream_t st = (hipStream_t)hip_stream;
    rc = run_direct_noalloc(c, st);
    if (rc) return rc;
    return finish_checks(c, st);
}

int fd_adjoint_gradient(const fd_grid* g, const float* vel, const fd_shot* shots, int nshots,
                        int ckpt_every, float* grad, void* workspace, size_t ws_bytes, void* hip_stream) {
    g_err.clear();
    if (!grad) return fail(FD_EINVAL, "grad is NULL");
    CallCtx c;
    int rc = prepare(c, g, vel, shots, nshots, 1, ckpt_every, workspace, ws_bytes);
    if (rc) return rc;
    c.grad = grad;
    hipStream_t st = (hipStream_t)hip_stream;
    rc = run_call(c, 1, st);
    if (rc) return rc;
    return finish_checks(c, st);
}

namespace {
int adjoint_opts(const fd_adjoint_opts* o, int* mode, int* K) {
    if (!o) return fail(FD_EINVAL, "opts is NULL");
    if (o->param < FD_PARAM_VELOCITY || o->param > FD_PARAM_M)
        return fail(FD_EINVAL, "unknown gradient parameter %d", o->param);
    if (o->ckpt == FD_CKPT_SEGMENT) {
        *mode = MODE_ADJ_SEGMENT;
        *K = o->ckpt_every;
    } else if (o->ckpt == FD_CKPT_REVOLVE) {
        *mode = MODE_ADJ_REVOLVE;
        *K = o->nsnap;
    } else {
        return fail(FD_EINVAL, "unknown checkpointing scheme %d", o->ckpt);
    }
    return FD_OK;
}
}  // namespace

int fd_adjoint_gradient_ex(const fd_grid* g, const float* vel, const fd_shot* shots, int nshots,
                           const fd_adjoint_opts* opts, float* grad, void* workspace, size_t ws_bytes,
                           void* hip_stream) {
    g_err.clear();
    int mode = 0, K = 0;
    int rc = adjoint_opts(opts, &mode, &K);
    if (rc) return rc;
    if (!grad) return fail(FD_EINVAL, "grad is NULL");
    CallCtx c;
    rc = prepare(c, g, vel, shots, nshots, mode, K, workspace, ws_bytes);
    if (rc) return rc;
    c.grad = grad;
    c.gparam = opts->param == FD_PARAM_SLOWNESS ? GP_SLOWNESS : opts->param == FD_PARAM_M ? GP_M : GP_VELOCITY;
    hipStream_t st = (hipStream_t)hip_stream;
    rc = run_call(c, mode, st);
    if (rc) return rc;
    return finish_checks(c, st);
}

size_t fd_adjoint_workspace_bytes(const fd_grid* g, const fd_shot* shots, int nshots, const fd_adjoint_opts* opts) {
    int mode = 0, K = 0;
    if (adjoint_opts(opts, &mode, &K) || check_grid(g) || !shots || nshots < 1) return 0;
    if (mode == MODE_ADJ_SEGMENT && (K < 1 || K > g->nt)) return 0;
    if (mode == MODE_ADJ_REVOLVE && (K < 0 || K > g->nt)) return 0;
    return make_layout(g, shots, nshots, mode, K).total;
}

int fd_revolve_plan(int nt, int nsnap, int* ops, long long max_ops, long long* nops, long long* fwd_steps) {
    g_err.clear();
    if (nt < 1) return fail(FD_EINVAL, "nt must be >= 1");
    if (nsnap < 0 || nsnap > nt) return fail(FD_EINVAL, "nsnap must be in [0, nt]");
    if (!nops) return fail(FD_EINVAL, "nops is NULL");
    RevolvePlanner p;
    const long long steps = p.plan(nt, nsnap);
    *nops = (long long)p.ops.size() / 2;
    if (fwd_steps) *fwd_steps = steps;
    if (ops) {
        if (max_ops < *nops) return fail(FD_ENOMEM, "plan has %lld ops, room for %lld", *nops, max_ops);
        std::memcpy(ops, p.ops.data(), sizeof(int) * p.ops.size());
    }
    return FD_OK;
}

int fd_error_norms(const float* num, const long long* num_stride, const float* ref, const long long* ref_stride,
                   const long long* n, double* out, void* workspace, size_t ws_bytes, void* hip_stream) {
    g_err.clear();
    if (!num || !ref || !num_stride || !ref_stride || !n || !out)
        return fail(FD_EINVAL, "num, ref, strides, n and out are required");
    for (int a = 0; a < 3; ++a)
        if (n[a] < 1) return fail(FD_EINVAL, "box extents must be >= 1");
    if (!workspace || ws_bytes < FD_ERROR_NORMS_WS_BYTES)
        return fail(FD_ENOMEM, "workspace must hold %d bytes", FD_ERROR_NORMS_WS_BYTES);
    if ((uintptr_t)workspace % 256) return fail(FD_EINVAL, "workspace must be 256-byte aligned");
    const long long total = n[0] * n[1] * n[2];
    const int nb = (int)std::min<long long>(kNormBlocks, (total + 255) / 256);
    launch_error_norms(num, num_stride, ref, ref_stride, n, (double*)workspace, nb, out, (hipStream_t)hip_stream);
    HIP_OK(hipGetLastError());
    return FD_OK;
}

size_t fd_dispersion_workspace_bytes(int nt, int nrec, int nscale) {
    if (nt < 2 || nrec < 1 || nscale < 0) return 0;
    return disp_layout(nt, nrec, nscale).total;
}

int fd_dispersion(const float* num, long long ld_num, const float* ref, long long ld_ref, int nt, int nrec,
                  double dt, int nscale, double omega0, float* gamma_dft, double* norm_dft, double* norm_cwt,
                  void* workspace, size_t ws_bytes, void* hip_stream) {
    g_err.clear();
    if (!num || !ref || !norm_dft) return fail(FD_EINVAL, "num, ref and norm_dft are required");
    if (nt < 2 || nrec < 1) return fail(FD_EINVAL, "need nt >= 2 and nrec >= 1");
    if (ld_num < nrec || ld_ref < nrec) return fail(FD_EINVAL, "row strides must be >= nrec");
    if (nscale < 0 || nscale > nt / 2) return fail(FD_EINVAL, "nscale must be in [0, nt/2]");
    if (norm_cwt && (nscale < 1 || !(dt > 0) || !(omega0 > 0)))
        return fail(FD_EINVAL, "the CWT norm needs nscale >= 1, dt > 0 and omega0 > 0");
    if (!workspace) return fail(FD_EINVAL, "workspace is NULL");
    if ((uintptr_t)workspace % 256) return fail(FD_EINVAL, "workspace must be 256-byte aligned");
    const int ns = norm_cwt ? nscale : 0;
    const DispLayout L = disp_layout(nt, nrec, ns);
    if (ws_bytes < L.total) return fail(FD_ENOMEM, "workspace too small: %zu < %zu bytes", ws_bytes, L.total);
    char* ws = (char*)workspace;
    hipStream_t st = (hipStream_t)hip_stream;
    const int R = disp_chunk(nt, nrec, ns);
    for (int r0 = 0; r0 < nrec; r0 += R) {
        const int rc = std::min(R, nrec - r0);
        FftPlan* fwd = nullptr;
        int rc2 = fft_plan(0, (size_t)nt, (size_t)rc, &fwd);
        if (rc2) return rc2;
        launch_rows_f64(num, ld_num, (double*)(ws + L.xa), nt, r0, rc, st);
        launch_rows_f64(ref, ld_ref, (double*)(ws + L.xb), nt, r0, rc, st);
        if ((rc2 = fft_run(fwd, ws + L.xa, ws + L.fa, st))) return rc2;
        if ((rc2 = fft_run(fwd, ws + L.xb, ws + L.fb, st))) return rc2;
        launch_gamma_dft(ws + L.fa, ws + L.fb, nt, rc, gamma_dft ? gamma_dft + (long long)r0 * nt : nullptr,
                         nt, norm_dft + r0, st);
        if (ns > 0) {
            FftPlan* inv = nullptr;
            if ((rc2 = fft_plan(1, (size_t)nt, (size_t)rc * ns, &inv))) return rc2;
            launch_cwt_spectra(ws + L.fa, nt, rc, ns, dt, omega0, ws + L.wa, st);
            launch_cwt_spectra(ws + L.fb, nt, rc, ns, dt, omega0, ws + L.wb, st);
            if ((rc2 = fft_run(inv, ws + L.wa, nullptr, st))) return rc2;
            if ((rc2 = fft_run(inv, ws + L.wb, nullptr, st))) return rc2;
            launch_gamma_cwt(ws + L.wa, ws + L.wb, nt, rc, ns, norm_cwt + r0, st);
        }
    }
    HIP_OK(hipGetLastError());
    return FD_OK;
}

}  // extern "C"
