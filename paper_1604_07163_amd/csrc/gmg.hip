// gmg.hip -- host side of the C ABI declared in include/gmg.h.
//
// Owns the multigrid hierarchy in HBM, schedules the V-cycle (grid-wide
// launches on fine levels, one persistent workgroup below the switch size) and
// drives preconditioned CG with every scalar (alpha, beta, norms, the stop
// flag) kept on the device.  The host only reads the stop flag every
// `check_every` iterations; kernels enqueued past convergence return at once.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <string>
#include <vector>

#include "gmg.h"
#include "kernels.hpp"

using gmg::bf16;
using gmg::ChebCoef;
using gmg::Lev;
using gmg::LevBuf;
using gmg::PcgState;
using gmg::Tiling;

namespace {

struct LevelHost {
    int n = 0, pitch = 0;
    long long plane = 0, nel = 0;  // nel = n * plane elements per array
    double s = 0;                  // h^-2
    double *kx64 = nullptr, *ky64 = nullptr, *kz64 = nullptr;
    bf16 *kx16 = nullptr, *ky16 = nullptr, *kz16 = nullptr;
    void *b = nullptr, *x = nullptr, *t1 = nullptr, *dinv = nullptr;
    bool g27 = false;           // Galerkin level: 27-point operator instead of links
    double lo = 0, hi = 0;      // Chebyshev interval of D^-1 A on this level
    ChebCoef<double> c64{};     // its coefficients, FP64 and FP32
    ChebCoef<float> c32{};
    double *a64 = nullptr;      // its 27 coefficient arrays (FP64, padded layout)
    void *av = nullptr;         // the same in the V-cycle type (== a64 in FP64 mode)
    Tiling til{};    // V-cycle stencil kernels
    Tiling til64{};  // FP64 outer operator (residual)
    Tiling til2{};   // FP64 outer apply, two points per lane
    int wx2 = 1;     // its waves along x (tiles of 128 wx2 x 4 / wx2 points)
    Tiling tilp{};   // pre-smoothing kernel, two rows per thread
    Tiling tilq{};   // one-sweep post-smoothing kernel
    Tiling tilr{};   // residual with z-reduction (even z-chunks)
    Tiling tilf{};   // pre-smoothing + residual in one sweep (64 x 8 tiles, even z-chunks)
    bool pre1 = false;   // pre-smoothing and residual in one sweep
    bool post1 = false;  // post-smoothing in one sweep, its result in t1 (else in x)
    gmg::Rows rows{};
    // the buffer that holds the level's V-cycle result after post-smoothing
    void *zout() const { return post1 ? t1 : x; }
};

}  // namespace

struct gmg_handle {
    gmg_options opt{};
    hipStream_t stream = nullptr;
    int L = 0;
    LevelHost lv[gmg::MAX_LEVELS];
    double *F = nullptr, *X = nullptr, *R = nullptr, *P = nullptr, *Q = nullptr;
    float *P32 = nullptr;  // MIXED: the search direction, stored in FP32
    double *partial = nullptr;
    double *partial2 = nullptr;   // first-stage sums of a large reduction (2 x NB_CHUNKS)
    int npartial = 0;
    PcgState *st = nullptr;       // device
    PcgState *st_in = nullptr;    // pinned host (uploads)
    PcgState *st_out = nullptr;   // pinned host (read-back)
    PcgState *cst = nullptr;      // device: inexact coarse CG (truncated hierarchy)
    PcgState *cst_out = nullptr;  // pinned host
    // device check of the last coefficients: tt = count of active links that
    // are not positive and finite, status = 3 if the coarsest operator is not
    // positive definite (read by gmg_create, and by every solve after
    // gmg_set_coefficients, which does not wait for it)
    PcgState *vst = nullptr;
    PcgState *vst_out = nullptr;  // pinned host
    hipEvent_t es0 = nullptr, es1 = nullptr;  // around the last gmg_set_coefficients
    bool setup_pending = false;   // its time is read at the next solve
    void *cp = nullptr, *cq = nullptr;  // coarse CG direction and A p (coarsest level, V type)
    long long coarse_its = 0;     // coarse CG iterations in the current solve
    double *chol = nullptr;       // coarsest factor, device
    int m = 0;
    void *dev_levels = nullptr;   // LevBuf<V,K>[L] on the device, then ChebCoef<V>[L] at dev_cheb
    void *dev_cheb = nullptr;
    int s_persist = 0;            // first level run by the persistent kernel (L-1 if none)
    bool persist = false;
    int persist_spread = 1;       // team packing stride (8 = one XCD) for persistent_wgs > 1
    int s2_persist = 0;           // first level on a single workgroup below a team (L-1: none)
    bool persist_lds = false;     // single-workgroup persistent levels staged in LDS
    size_t lds_bytes = 0;         // its dynamic LDS size
    gmg::GridBar *bar = nullptr;  // device barrier of the persistent team
    hipEvent_t ev0 = nullptr, ev1 = nullptr;
    std::vector<void *> allocs;   // device buffers to free (none for a static-workspace handle)
    char err[256] = "";           // last error message (fixed storage: setting it allocates nothing)
    // static workspace (gmg_solve_static): buffers are carved from `arena`
    // instead of allocated, and no event, pinned buffer or heap object is made
    char *arena = nullptr;
    size_t arena_cap = 0, arena_used = 0;
    double setup_ms = 0;
    // kernel timing: event pairs per kernel class
    bool prof_on = false;
    std::vector<hipEvent_t> prof_ev[GMG_K_COUNT];
    int prof_used[GMG_K_COUNT] = {};
};

namespace {

// The static workspace of gmg_solve_static (see there).
constexpr size_t kStaticBytes = 64ull << 20;  // holds the hierarchy of a 65^3 grid in either precision
constexpr int kMaxDevices = 64;
static __device__ __align__(256) unsigned char scratch[kStaticBytes];
void *g_scratch[kMaxDevices];  // address of `scratch` on each device
gmg_handle g_static_handle[kMaxDevices];
PcgState g_static_state[kMaxDevices][4];  // st_in, st_out, cst_out, vst_out (pageable host memory)
int g_static_last_device = 0;

gmg_status fail(gmg_handle *h, gmg_status s, const char *fmt, ...) __attribute__((format(printf, 3, 4)));
gmg_status fail(gmg_handle *h, gmg_status s, const char *fmt, ...) {
    if (h) {
        va_list ap;
        va_start(ap, fmt);
        vsnprintf(h->err, sizeof(h->err), fmt, ap);
        va_end(ap);
    }
    return s;
}

#define HIPCHK(call)                                                                           \
    do {                                                                                       \
        hipError_t e_ = (call);                                                                \
        if (e_ != hipSuccess)                                                                  \
            return fail(h, GMG_ERR_HIP, "%s: %s", #call, hipGetErrorString(e_));                  \
    } while (0)
#define LAUNCHCHK()                                                                            \
    do {                                                                                       \
        hipError_t e_ = hipGetLastError();                                                     \
        if (e_ != hipSuccess)                                                                  \
            return fail(h, GMG_ERR_HIP, "kernel launch: %s", hipGetErrorString(e_));              \
    } while (0)
#define STCHK(expr)                   \
    do {                              \
        gmg_status s_ = (expr);       \
        if (s_ != GMG_OK) return s_;  \
    } while (0)

int round_up(int a, int b) { return (a + b - 1) / b * b; }
unsigned blocks_for(long long n, int nt) { return (unsigned)((n + nt - 1) / nt); }

// Workgroup-count targets of the z-marching stencil kernels (the z-chunk
// length follows from them, at least kMinChunk planes).  Measured on MI355X:
// 8-9 plane chunks stream best in FP64 and FP32 alike (at 1025^3 the MIXED
// V-cycle kernels ran 15 % faster than with one chunk per column).  Levels
// too small to give kMinWorkgroups workgroups that way take shorter chunks,
// down to one plane: there a kernel is bound by the latency of its z-march
// (129^3 .. 33^3 levels: a MIXED V-cycle at 257^3 8 % faster, 513^3 1.5 %).
int env_int(const char *name, int dflt) {
    const char *e = getenv(name);
    const int v = e ? atoi(e) : 0;
    return v > 0 ? v : dflt;
}

constexpr int kMinChunk = 8;
constexpr int kMinWorkgroups = 1024;

// width: x extent of a tile (TX, or TX2 for the two-points-per-lane apply);
// rows: y extent (TY, or TY_PRE for the two-rows-per-thread pre-smoothing)
// min_chunk: shortest z-chunk while kMinWorkgroups are launched anyway;
// pad8: round the tile rows up to a multiple of 8 (empty tiles exit at once)
// so that the XCD y-slab order of tile_of applies.
Tiling make_tiling(int n, int target, int width = gmg::TX, int rows = gmg::TY, int min_chunk = kMinChunk,
                   bool pad8 = false) {
    Tiling t;
    t.tiles_x = (n - 2) / width + 1;  // covers i = 0 .. n-2
    t.tiles_y = (n - 2 + rows - 1) / rows;
    if (pad8) t.tiles_y = (t.tiles_y + 7) & ~7;
    const int planes = n - 2;
    const int tiles = t.tiles_x * t.tiles_y;
    int nch = (target + tiles - 1) / tiles;
    if (nch > planes / min_chunk) nch = planes / min_chunk;
    // small levels: too few workgroups to hide the latency of a long z-march,
    // so chunks shorten (down to one plane) until kMinWorkgroups are launched
    if ((long long)tiles * nch < kMinWorkgroups) nch = std::min(planes, (kMinWorkgroups + tiles - 1) / tiles);
    if (nch < 1) nch = 1;
    t.zchunk = (planes + nch - 1) / nch;
    nch = (planes + t.zchunk - 1) / t.zchunk;
    t.nblocks = t.tiles_x * t.tiles_y * nch;
    return t;
}

// A tiling with z-chunks of `chunk` planes, shortened (down to one plane)
// where that would launch fewer than kMinWorkgroups workgroups.
Tiling chunk_tiling(int n, int chunk, int width, int rows) {
    // the one-sweep kernels address a chunk by 32-bit buffer offsets from its
    // lowest halo plane: the chunk with its halo and look-ahead planes (at
    // most zchunk + 7 planes of 8-byte elements, zchunk possibly made even)
    // stays below 2^31 bytes (check_options rejects n where 1 plane cannot)
    const long long plane_bytes = 8LL * n * round_up(n, 64);
    chunk = (int)std::min<long long>(chunk, std::max(1LL, 0x7fffffffLL / plane_bytes - 8));
    Tiling t;
    t.tiles_x = (n - 2) / width + 1;
    t.tiles_y = (n - 2 + rows - 1) / rows;
    const int planes = n - 2, tiles = t.tiles_x * t.tiles_y;
    int nch = (planes + chunk - 1) / chunk;
    if ((long long)tiles * nch < kMinWorkgroups) nch = std::min(planes, (kMinWorkgroups + tiles - 1) / tiles);
    t.zchunk = (planes + nch - 1) / nch;
    nch = (planes + t.zchunk - 1) / t.zchunk;
    t.nblocks = t.tiles_x * t.tiles_y * nch;
    return t;
}

// The same tiling with an even number of planes per z-chunk (so every chunk
// starts on an odd plane), for the residual with z-reduction.
Tiling even_chunks(Tiling t, int n) {
    const int planes = n - 2;
    t.zchunk += t.zchunk & 1;
    const int nch = (planes + t.zchunk - 1) / t.zchunk;
    t.nblocks = t.tiles_x * t.tiles_y * nch;
    return t;
}

// Prolongation grid: one thread per coarse cell (I,J,K), I,J,K in 0..nc-2.
dim3 prolong_grid(int nc) {
    return dim3((unsigned)((nc - 1 + gmg::TX - 1) / gmg::TX), (unsigned)((nc - 1 + gmg::TY - 1) / gmg::TY),
                (unsigned)(nc - 1));
}

gmg::Rows make_rows(int n, int pitch, long long plane) {
    gmg::Rows r;
    r.n = n;
    r.pitch = pitch;
    r.plane = plane;
    r.half_w = n / 2;  // pairs cover x = 0 .. 2*half_w-1 (>= n-2, <= pitch)
    const long long nrows = (long long)(n - 2) * (n - 2);
    int l = 0;
    while ((1 << l) < r.half_w && (1 << l) < gmg::NT_FLAT) ++l;
    r.tpr_log2 = l;
    if (r.half_w >= gmg::NT_FLAT) {
        r.segs = (r.half_w + gmg::NT_FLAT - 1) / gmg::NT_FLAT;
        r.nblocks = (int)(nrows * r.segs);
    } else {
        r.segs = 0;
        const int rpb = gmg::NT_FLAT >> l;
        r.nblocks = (int)((nrows + rpb - 1) / rpb);
    }
    return r;
}

// A zero-filled device buffer of `count` elements: hipMalloc'd (freed by
// gmg_destroy), or, for a static-workspace handle, the next 256-byte aligned
// piece of the arena (zeroed in one pass once every piece is assigned).
template <typename T>
gmg_status dalloc(gmg_handle *h, T **p, long long count) {
    const size_t bytes = (size_t)count * sizeof(T);
    if (h->arena) {
        const size_t off = (h->arena_used + 255) & ~(size_t)255;
        if (off + bytes > h->arena_cap)
            return fail(h, GMG_ERR_DIMS, "the hierarchy needs more than the %zu-byte static workspace", h->arena_cap);
        *p = (T *)(h->arena + off);
        h->arena_used = off + bytes;
        return GMG_OK;
    }
    void *q = nullptr;
    hipError_t e = hipMalloc(&q, bytes);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        return fail(h, GMG_ERR_NOMEM, "hipMalloc of %zu bytes failed", bytes);
    }
    h->allocs.push_back(q);
    e = hipMemsetAsync(q, 0, bytes, h->stream);
    if (e != hipSuccess) return fail(h, GMG_ERR_HIP, "hipMemsetAsync failed");
    *p = (T *)q;
    return GMG_OK;
}

bool mixed(const gmg_handle *h) { return h->opt.precision == GMG_MIXED; }

template <typename K>
struct KSel;
template <>
struct KSel<double> {
    static const double *x(const LevelHost &l) { return l.kx64; }
    static const double *y(const LevelHost &l) { return l.ky64; }
    static const double *z(const LevelHost &l) { return l.kz64; }
};
template <>
struct KSel<bf16> {
    static const bf16 *x(const LevelHost &l) { return l.kx16; }
    static const bf16 *y(const LevelHost &l) { return l.ky16; }
    static const bf16 *z(const LevelHost &l) { return l.kz16; }
};

template <typename V, typename K>
Lev<V, K> view(const LevelHost &l) {
    Lev<V, K> v;
    v.n = l.n;
    v.pitch = l.pitch;
    v.plane = l.plane;
    v.s = (V)l.s;
    v.kx = KSel<K>::x(l);
    v.ky = KSel<K>::y(l);
    v.kz = KSel<K>::z(l);
    v.dinv = (const V *)l.dinv;
    v.a27 = l.g27 ? (const V *)l.av : nullptr;
    v.nel = l.nel;
    return v;
}

template <typename V>
const ChebCoef<V> &cheb(const gmg_handle *h, int l);
template <>
const ChebCoef<double> &cheb<double>(const gmg_handle *h, int l) { return h->lv[l].c64; }
template <>
const ChebCoef<float> &cheb<float>(const gmg_handle *h, int l) { return h->lv[l].c32; }

// Chebyshev-Jacobi coefficients for the interval [lo, hi] of D^-1 A (three-term
// recurrence of the Chebyshev iteration, Saad Alg. 12.1).
void set_cheb(LevelHost &lh, int degree, double lo, double hi) {
    const double theta = 0.5 * (hi + lo), delta = 0.5 * (hi - lo);
    const double sigma = theta / delta;
    ChebCoef<double> c{};
    c.m = degree;
    c.cfirst = 1.0 / theta;
    double rho = 1.0 / sigma;
    for (int j = 1; j < c.m; ++j) {
        const double rn = 1.0 / (2.0 * sigma - rho);
        c.c1[j] = rn * rho;
        c.c2[j] = 2.0 * rn / delta;
        rho = rn;
    }
    lh.lo = lo;
    lh.hi = hi;
    lh.c64 = c;
    lh.c32 = ChebCoef<float>{};
    lh.c32.m = c.m;
    lh.c32.cfirst = (float)c.cfirst;
    for (int j = 0; j < gmg::MAX_DEGREE; ++j) {
        lh.c32.c1[j] = (float)c.c1[j];
        lh.c32.c2[j] = (float)c.c2[j];
    }
}

// ------------------------------------------------------------------ kernel timing
// Brackets one launch with HIP events on the handle's stream when profiling
// is on and `on` holds (finest-level launches and the coarse-level kernels).
constexpr int kProfMax = 1 << 15;
struct Prof {
    gmg_handle *h;
    int cls, idx = -1;
    Prof(gmg_handle *h_, int c, bool on) : h(h_), cls(c) {
        if (!on || !h->prof_on) return;
        std::vector<hipEvent_t> &v = h->prof_ev[c];
        const int i = h->prof_used[c];
        if (i >= kProfMax) return;
        if ((int)v.size() < 2 * (i + 1)) {
            hipEvent_t a, b;
            if (hipEventCreate(&a) != hipSuccess) return;
            if (hipEventCreate(&b) != hipSuccess) {
                (void)hipEventDestroy(a);
                return;
            }
            v.push_back(a);
            v.push_back(b);
        }
        if (hipEventRecord(v[2 * i], h->stream) != hipSuccess) return;
        idx = i;
    }
    ~Prof() {
        if (idx < 0) return;
        if (hipEventRecord(h->prof_ev[cls][2 * idx + 1], h->stream) == hipSuccess) h->prof_used[cls] = idx + 1;
    }
};

gmg_status finalize(gmg_handle *h, int count, int stage, PcgState *state = nullptr);
gmg_status coefficient_status(gmg_handle *h, const PcgState &v);

// ------------------------------------------------------------------ smoothing
// Chebyshev-Jacobi smoothing on a Galerkin level: the recurrence and buffer
// rotation of smooth_grid with the 27-point operator, whose centre
// coefficient is the Jacobi diagonal.
template <typename V, typename K>
gmg_status smooth27(gmg_handle *h, int l, bool from_zero, const int *skip) {
    LevelHost &lh = h->lv[l];
    const ChebCoef<V> &cc = cheb<V>(h, l);
    V *bufs[2] = {(V *)lh.x, (V *)lh.t1};
    V *b = (V *)lh.b;
    const V *a = (const V *)lh.av;
    const dim3 grid(lh.til.nblocks), blk(gmg::NT);
    int cur, prev;
    if (from_zero) {
        V *dst = cc.m == 1 ? bufs[0] : bufs[1];
        gmg::k_cheb_first<V, K, false><<<grid, blk, 0, h->stream>>>(view<V, K>(lh), lh.til, b, nullptr, nullptr, dst,
                                                                     cc.cfirst, skip);
        LAUNCHCHK();
        if (cc.m == 1) return GMG_OK;
        cur = 1;
        prev = -1;
    } else {
        gmg::k_sweep27<V, 2, 0><<<grid, blk, 0, h->stream>>>(lh.n, lh.pitch, lh.plane, lh.til, a, lh.nel, b, bufs[0],
                                                              nullptr, bufs[1], V(0), cc.cfirst, skip);
        LAUNCHCHK();
        cur = 1;
        prev = 0;
    }
    for (int j = 1; j < cc.m; ++j) {
        const int dst = 1 - cur;
        if (prev < 0)
            gmg::k_sweep27<V, 2, 1><<<grid, blk, 0, h->stream>>>(lh.n, lh.pitch, lh.plane, lh.til, a, lh.nel, b,
                                                                  bufs[cur], nullptr, bufs[dst], cc.c1[j], cc.c2[j],
                                                                  skip);
        else
            gmg::k_sweep27<V, 2, 2><<<grid, blk, 0, h->stream>>>(lh.n, lh.pitch, lh.plane, lh.til, a, lh.nel, b,
                                                                  bufs[cur], bufs[prev], bufs[dst], cc.c1[j],
                                                                  cc.c2[j], skip);
        LAUNCHCHK();
        prev = cur;
        cur = dst;
    }
    if (cur != 0) {
        gmg::k_cast<V, V><<<gmg::NB_FLAT, gmg::NT_FLAT, 0, h->stream>>>(lh.nel, bufs[1], bufs[0], skip);
        LAUNCHCHK();
    }
    return GMG_OK;
}

// Chebyshev-Jacobi smoothing of A_l x = b_l on the grid path.  The iterate
// alternates between x and t1 (x_{j+1} overwrites the buffer of x_{j-1});
// odd degrees end with a copy into x.  `dot_r64` (finest level, post-smoothing
// only) fuses the partial sums of r.z into the last sweep; returns the number
// of partials written (0 if none).
template <typename V, typename K>
gmg_status smooth_grid(gmg_handle *h, int l, bool from_zero, const double *r64_cvt, const double *dot_r64,
                       const int *skip, int *nparts, const double *dot_q64 = nullptr) {
    LevelHost &lh = h->lv[l];
    if (lh.g27) {  // never the finest level: no conversion, no fused dot
        if (nparts) *nparts = 0;
        return smooth27<V, K>(h, l, from_zero, skip);
    }
    const Lev<V, K> L = view<V, K>(lh);
    const ChebCoef<V> &cc = cheb<V>(h, l);
    V *bufs[2] = {(V *)lh.x, (V *)lh.t1};
    V *b = (V *)lh.b;
    const dim3 grid(lh.til.nblocks), blk(gmg::NT);
    int cur, prev;
    if (nparts) *nparts = 0;
    const bool fin = l == 0;
    if (from_zero && !r64_cvt && cc.m >= 2) {
        // x1 and x2 in one sweep; x1 is stored only when a third step needs it
        Prof pf(h, GMG_K_CHEB_PRE2, fin);
        const dim3 gp(lh.tilp.nblocks);
        if (cc.m == 2)
            gmg::k_cheb_pre2<V, K, false><<<gp, blk, 0, h->stream>>>(L, lh.tilp, b, bufs[0], nullptr, cc.cfirst,
                                                                      cc.c1[1], cc.c2[1], skip);
        else
            gmg::k_cheb_pre2<V, K, true><<<gp, blk, 0, h->stream>>>(L, lh.tilp, b, bufs[0], bufs[1], cc.cfirst,
                                                                     cc.c1[1], cc.c2[1], skip);
        LAUNCHCHK();
        cur = 0;
        prev = 1;
        for (int j = 2; j < cc.m; ++j) {
            const int dst = 1 - cur;
            Prof pf2(h, GMG_K_CHEB_STEP_PREV, fin);
            gmg::k_cheb_step<V, K, 2, false><<<grid, blk, 0, h->stream>>>(L, lh.til, b, bufs[cur], bufs[prev], bufs[dst],
                                                                            cc.c1[j], cc.c2[j], nullptr, nullptr, skip);
            LAUNCHCHK();
            prev = cur;
            cur = dst;
        }
        if (cur != 0) {
            gmg::k_cast<V, V><<<gmg::NB_FLAT, gmg::NT_FLAT, 0, h->stream>>>(lh.nel, bufs[1], bufs[0], skip);
            LAUNCHCHK();
        }
        return GMG_OK;
    }
    if (from_zero) {
        V *dst = cc.m == 1 ? bufs[0] : bufs[1];
        Prof pf(h, GMG_K_CHEB_FIRST, fin);
        if (r64_cvt)
            gmg::k_cheb_first<V, K, true><<<grid, blk, 0, h->stream>>>(L, lh.til, nullptr, r64_cvt, b, dst, cc.cfirst,
                                                                        skip);
        else
            gmg::k_cheb_first<V, K, false><<<grid, blk, 0, h->stream>>>(L, lh.til, b, nullptr, nullptr, dst, cc.cfirst,
                                                                         skip);
        LAUNCHCHK();
        if (cc.m == 1) return GMG_OK;
        cur = 1;
        prev = -1;
    } else if (lh.post1) {
        // both steps in one sweep, x0 in x, the result in t1
        Prof pf(h, GMG_K_CHEB_POST2, fin);
        constexpr int rows = gmg::TY_POST;
        const dim3 gq(lh.tilq.nblocks), bq(gmg::TX * rows);
        const V c0 = cc.cfirst, c1 = cc.c1[1], c2 = cc.c2[1];
        if (dot_r64 && dot_q64)
            gmg::k_post2<V, K, 2, rows><<<gq, bq, 0, h->stream>>>(L, lh.tilq, b, bufs[0], bufs[1], c0, c1, c2,
                                                                   dot_r64, h->partial, skip, dot_q64);
        else if (dot_r64)
            gmg::k_post2<V, K, 1, rows><<<gq, bq, 0, h->stream>>>(L, lh.tilq, b, bufs[0], bufs[1], c0, c1, c2,
                                                                   dot_r64, h->partial, skip);
        else
            gmg::k_post2<V, K, 0, rows><<<gq, bq, 0, h->stream>>>(L, lh.tilq, b, bufs[0], bufs[1], c0, c1, c2,
                                                                   nullptr, nullptr, skip);
        if (dot_r64 && nparts) *nparts = lh.tilq.nblocks;
        LAUNCHCHK();
        return GMG_OK;
    } else {
        Prof pf(h, GMG_K_CHEB_STEP, fin);
        gmg::k_cheb_step<V, K, 0, false><<<grid, blk, 0, h->stream>>>(L, lh.til, b, bufs[0], nullptr, bufs[1], V(0),
                                                                        cc.cfirst, nullptr, nullptr, skip);
        LAUNCHCHK();
        cur = 1;
        prev = 0;
    }
    for (int j = 1; j < cc.m; ++j) {
        const int dst = 1 - cur;
        const bool fuse = dot_r64 && (j == cc.m - 1) && dst == 0;
        Prof pf(h, prev < 0 ? GMG_K_CHEB_STEP : fuse ? GMG_K_CHEB_STEP_DOT : GMG_K_CHEB_STEP_PREV, fin);
        if (prev < 0) {
            gmg::k_cheb_step<V, K, 1, false><<<grid, blk, 0, h->stream>>>(L, lh.til, b, bufs[cur], nullptr, bufs[dst],
                                                                            cc.c1[j], cc.c2[j], nullptr, nullptr, skip);
        } else if (fuse) {
            gmg::k_cheb_step<V, K, 2, true><<<grid, blk, 0, h->stream>>>(L, lh.til, b, bufs[cur], bufs[prev], bufs[dst],
                                                                           cc.c1[j], cc.c2[j], dot_r64, h->partial, skip,
                                                                           dot_q64);
            if (nparts) *nparts = lh.til.nblocks;
        } else {
            gmg::k_cheb_step<V, K, 2, false><<<grid, blk, 0, h->stream>>>(L, lh.til, b, bufs[cur], bufs[prev], bufs[dst],
                                                                            cc.c1[j], cc.c2[j], nullptr, nullptr, skip);
        }
        LAUNCHCHK();
        prev = cur;
        cur = dst;
    }
    if (cur != 0) {
        gmg::k_cast<V, V><<<gmg::NB_FLAT, gmg::NT_FLAT, 0, h->stream>>>(lh.nel, bufs[1], bufs[0], skip);
        LAUNCHCHK();
    }
    if (dot_r64 && nparts && *nparts == 0) {
        gmg::k_dot<V><<<lh.rows.nblocks, gmg::NT_FLAT, 0, h->stream>>>(lh.rows, dot_r64, bufs[0], h->partial, skip);
        LAUNCHCHK();
        if (dot_q64) {
            gmg::k_dot<V><<<lh.rows.nblocks, gmg::NT_FLAT, 0, h->stream>>>(lh.rows, dot_q64, bufs[0],
                                                                            h->partial + lh.rows.nblocks, skip);
            LAUNCHCHK();
        }
        *nparts = lh.rows.nblocks;
    }
    return GMG_OK;
}

// Inexact coarsest solve of a truncated hierarchy: Jacobi-CG on grid-wide
// launches, its scalars on the device; the host polls the stop flag every 8
// iterations (the coarse solve of the truncation strategy pays these launches
// and reductions on every V-cycle).
template <typename V, typename K>
gmg_status coarse_cg(gmg_handle *h, const int *skip) {
    LevelHost &c = h->lv[h->L - 1];
    const int *cskip = &h->cst->done;
    gmg::k_cg_begin<<<1, 64, 0, h->stream>>>(h->cst, skip, h->opt.coarse_rtol * h->opt.coarse_rtol,
                                             h->opt.coarse_max_it);
    LAUNCHCHK();
    gmg::k_cg_start<V><<<c.rows.nblocks, gmg::NT_FLAT, 0, h->stream>>>(c.rows, (const V *)c.b, (V *)c.x, (V *)c.t1,
                                                                        (V *)h->cp, (const V *)c.dinv, h->partial, cskip);
    LAUNCHCHK();
    STCHK(finalize(h, c.rows.nblocks, gmg::ST_C_INIT, h->cst));
    for (int chunk = 0; chunk * 8 < h->opt.coarse_max_it + 8; ++chunk) {
        for (int i = 0; i < 8; ++i) {
            if (c.g27)
                gmg::k_sweep27<V, 0, 0, true><<<c.til.nblocks, gmg::NT, 0, h->stream>>>(
                    c.n, c.pitch, c.plane, c.til, (const V *)c.av, c.nel, nullptr, (const V *)h->cp, nullptr,
                    (V *)h->cq, V(0), V(0), cskip, h->partial);
            else
                gmg::k_apply<V, K, true><<<c.til.nblocks, gmg::NT, 0, h->stream>>>(
                    view<V, K>(c), c.til, (const V *)h->cp, (V *)h->cq, h->partial, cskip);
            LAUNCHCHK();
            STCHK(finalize(h, c.til.nblocks, gmg::ST_C_ALPHA, h->cst));
            gmg::k_cg_update<V><<<c.rows.nblocks, gmg::NT_FLAT, 0, h->stream>>>(
                c.rows, (V *)c.x, (V *)c.t1, (const V *)h->cp, (const V *)h->cq, (const V *)c.dinv, h->cst, h->partial);
            LAUNCHCHK();
            STCHK(finalize(h, c.rows.nblocks, gmg::ST_C_RR, h->cst));
            gmg::k_cg_p<V><<<c.rows.nblocks, gmg::NT_FLAT, 0, h->stream>>>(c.rows, (const V *)c.t1, (V *)h->cp,
                                                                          (const V *)c.dinv, h->cst);
            LAUNCHCHK();
        }
        HIPCHK(hipMemcpyAsync(h->cst_out, h->cst, sizeof(PcgState), hipMemcpyDeviceToHost, h->stream));
        HIPCHK(hipStreamSynchronize(h->stream));
        if (h->cst_out->done) break;
    }
    h->coarse_its += h->cst_out->its;
    return GMG_OK;
}

// b_{l+1} = R (b_l - A_l x_l): the residual into t1 (free between pre- and
// post-smoothing), then full weighting onto the coarse right-hand side.
template <typename V, typename K>
gmg_status residual_restrict(gmg_handle *h, int l, const int *skip) {
    LevelHost &f = h->lv[l], &c = h->lv[l + 1];
    {
        Prof pf(h, GMG_K_LEVEL_RESIDUAL, l == 0);
        if (f.g27)
            gmg::k_sweep27<V, 1, 0><<<f.til.nblocks, gmg::NT, 0, h->stream>>>(
                f.n, f.pitch, f.plane, f.til, (const V *)f.av, f.nel, (const V *)f.b, (const V *)f.x, nullptr,
                (V *)f.t1, V(0), V(0), skip);
        else  // z-sums of the residual at the coarse planes, into t1
            gmg::k_residual_zr<V, K><<<f.tilr.nblocks, gmg::NT, 0, h->stream>>>(view<V, K>(f), f.tilr,
                                                                               (const V *)f.b, (const V *)f.x,
                                                                               (V *)f.t1, skip);
        LAUNCHCHK();
    }
    Prof pf(h, GMG_K_RESTRICT, l == 0);
    if (f.g27)
        gmg::k_restrict<V><<<c.til.nblocks, gmg::NT, 0, h->stream>>>(c.n, c.pitch, c.plane, c.til, f.pitch, f.plane,
                                                                     (const V *)f.t1, (V *)c.b, skip);
    else
        gmg::k_restrict_xy<V><<<c.til.nblocks, gmg::NT, 0, h->stream>>>(c.n, c.pitch, c.plane, c.til, f.pitch,
                                                                        f.plane, (const V *)f.t1, (V *)c.b, skip);
    LAUNCHCHK();
    return GMG_OK;
}

// Pre-smoothing from zero and the residual's z-sums in one sweep (x2 into x,
// the z-sums into t1), then the in-plane restriction to the coarse b.
template <typename V, typename K>
gmg_status pre_residual_restrict(gmg_handle *h, int l, const int *skip) {
    LevelHost &f = h->lv[l], &c = h->lv[l + 1];
    const ChebCoef<V> &cc = cheb<V>(h, l);
    {
        Prof pf(h, GMG_K_PRE2_RES, l == 0);
        constexpr int rows = gmg::TY_PRE_RES;
        gmg::k_pre2_res<V, K, rows><<<f.tilf.nblocks, gmg::TX * rows, 0, h->stream>>>(
            view<V, K>(f), f.tilf, (const V *)f.b, (V *)f.x, (V *)f.t1, cc.cfirst, cc.c1[1], cc.c2[1], skip);
        LAUNCHCHK();
    }
    Prof pf(h, GMG_K_RESTRICT, l == 0);
    gmg::k_restrict_xy<V><<<c.til.nblocks, gmg::NT, 0, h->stream>>>(c.n, c.pitch, c.plane, c.til, f.pitch, f.plane,
                                                                    (const V *)f.t1, (V *)c.b, skip);
    LAUNCHCHK();
    return GMG_OK;
}

template <typename V, typename K>
gmg_status coarse_part(gmg_handle *h, const int *skip) {
    const int last = h->L - 1;
    if (h->opt.coarse_solver == 1) return coarse_cg<V, K>(h, skip);
    Prof pf(h, h->persist ? GMG_K_PERSISTENT : GMG_K_COARSE_SOLVE, true);
    if (h->persist && h->opt.persistent_wgs == 1 && h->persist_lds) {
        gmg::k_persistent_lds<V, K><<<1, gmg::NT_PERSIST, h->lds_bytes, h->stream>>>(
            (const LevBuf<V, K> *)h->dev_levels, (const ChebCoef<V> *)h->dev_cheb, h->s_persist, last, h->chol, h->m,
            skip);
    } else if (h->persist && h->opt.persistent_wgs == 1) {
        gmg::k_persistent<V, K><<<1, gmg::NT_PERSIST, 0, h->stream>>>((const LevBuf<V, K> *)h->dev_levels,
                                                                       (const ChebCoef<V> *)h->dev_cheb, h->s_persist,
                                                                       last, h->chol, h->m, skip, nullptr, 1, 1, 0);
    } else if (h->persist) {
        // A team of co-resident workgroups (cooperative launch: an error, never
        // a hang, if they cannot all be resident).  With a second switch level the
        // team runs the middle levels and one workgroup the ones below it.
        const LevBuf<V, K> *lv = (const LevBuf<V, K> *)h->dev_levels;
        const ChebCoef<V> *cc = (const ChebCoef<V> *)h->dev_cheb;
        const int s2 = h->s2_persist;
        int s0 = h->s_persist, la = s2 < last ? s2 : last, m = h->m, na = h->opt.persistent_wgs,
            sp = h->persist_spread, ph = s2 < last ? 1 : 0;
        const double *lf = h->chol;
        gmg::GridBar *bar = h->bar;
        void *args[] = {&lv, &cc, &s0, &la, &lf, &m, &skip, &bar, &na, &sp, &ph};
        HIPCHK(hipLaunchCooperativeKernel((const void *)gmg::k_persistent<V, K>, dim3(na * sp), dim3(gmg::NT_PERSIST),
                                          args, 0, h->stream));
        if (s2 < last) {
            gmg::k_persistent<V, K><<<1, gmg::NT_PERSIST, 0, h->stream>>>(lv, cc, s2, last, h->chol, h->m, skip,
                                                                           nullptr, 1, 1, 0);
            LAUNCHCHK();
            ph = 2;
            HIPCHK(hipLaunchCooperativeKernel((const void *)gmg::k_persistent<V, K>, dim3(na * sp),
                                              dim3(gmg::NT_PERSIST), args, 0, h->stream));
        }
    } else {
        const LevelHost &c = h->lv[last];
        gmg::k_coarse_solve<V><<<1, 256, 0, h->stream>>>(c.n, c.pitch, c.plane, h->m, h->chol, (const V *)c.b,
                                                          (V *)c.x, skip);
    }
    LAUNCHCHK();
    return GMG_OK;
}

// z = B r: one V-cycle on the FP64 residual r (= h->R).  The result is in
// lv[0].x (FP64 or FP32).  With want_dot, partial sums of r.z are left in
// h->partial and their count in *nparts.
template <typename V, typename K>
gmg_status vcycle(gmg_handle *h, const int *skip, bool want_dot, int *nparts, bool b_ready = false) {
    const int last = h->L - 1;
    const bool mx = mixed(h);
    if (nparts) *nparts = 0;
    if (last == 0) {  // the finest level is the coarsest: exact solve
        LevelHost &l0 = h->lv[0];
        if (mx) {
            gmg::k_cast<double, V><<<gmg::NB_FLAT, gmg::NT_FLAT, 0, h->stream>>>(l0.nel, h->R, (V *)l0.b, skip);
            LAUNCHCHK();
        }
        STCHK((coarse_part<V, K>(h, skip)));
        if (want_dot) {
            gmg::k_dot<V><<<l0.rows.nblocks, gmg::NT_FLAT, 0, h->stream>>>(l0.rows, h->R, (const V *)l0.x, h->partial,
                                                                            skip);
            LAUNCHCHK();
            if (h->opt.flexible) {
                gmg::k_dot<V><<<l0.rows.nblocks, gmg::NT_FLAT, 0, h->stream>>>(l0.rows, h->Q, (const V *)l0.x,
                                                                                h->partial + l0.rows.nblocks, skip);
                LAUNCHCHK();
            }
            *nparts = l0.rows.nblocks;
        }
        return GMG_OK;
    }
    const int s = h->s_persist;  // levels 0..s-1 on the grid path
    for (int l = 0; l < s; ++l) {
        const double *cvt = (l == 0 && mx && !b_ready) ? h->R : nullptr;
        if (h->lv[l].pre1 && !cvt) {
            STCHK((pre_residual_restrict<V, K>(h, l, skip)));
        } else {
            STCHK((smooth_grid<V, K>(h, l, true, cvt, nullptr, skip, nullptr)));
            STCHK((residual_restrict<V, K>(h, l, skip)));
        }
    }
    STCHK((coarse_part<V, K>(h, skip)));
    for (int l = s - 1; l >= 0; --l) {
        LevelHost &f = h->lv[l], &c = h->lv[l + 1];
        {
            Prof pf(h, GMG_K_PROLONG, l == 0);
            gmg::k_prolong<V><<<prolong_grid(c.n), gmg::NT, 0, h->stream>>>(f.pitch, f.plane, c.n, c.pitch, c.plane,
                                                                            (const V *)c.zout(), (V *)f.x, skip);
            LAUNCHCHK();
        }
        STCHK((smooth_grid<V, K>(h, l, false, nullptr, (l == 0 && want_dot) ? h->R : nullptr, skip,
                                 l == 0 ? nparts : nullptr,
                                 (l == 0 && want_dot && h->opt.flexible) ? h->Q : nullptr)));
    }
    return GMG_OK;
}

// b_ready: MIXED only -- the FP32 finest right-hand side was already written
// from r (by k_update_r), so the first sweep need not convert r.
gmg_status vcycle_any(gmg_handle *h, const int *skip, bool want_dot, int *nparts, bool b_ready = false) {
    return mixed(h) ? vcycle<float, bf16>(h, skip, want_dot, nparts, b_ready)
                    : vcycle<double, double>(h, skip, want_dot, nparts);
}

// Sums `count` per-workgroup partials (two arrays for the paired stages) into
// the PCG state.  Above kChunkedFrom partials a first stage spreads the loads
// over NB_CHUNKS workgroups (a single workgroup summing 2.6e5 partials, the
// row kernels' count at 513^3, takes 50 us).
constexpr int kChunkedFrom = 4096;
gmg_status finalize(gmg_handle *h, int count, int stage, PcgState *state) {
    PcgState *st = state ? state : h->st;
    const double *src = h->partial;
    if (count > kChunkedFrom) {
        const bool two = stage == gmg::ST_BETA_FLEX || stage == gmg::ST_C_INIT || stage == gmg::ST_C_RR;
        const bool gated = !(stage == gmg::ST_BB || stage == gmg::ST_RR0 || stage == gmg::ST_RHO0 ||
                             stage == gmg::ST_TT);
        const int chunk = (count + gmg::NB_CHUNKS - 1) / gmg::NB_CHUNKS;
        const int nb = (count + chunk - 1) / chunk;
        gmg::k_reduce_chunks<<<nb, 256, 0, h->stream>>>(h->partial, count, chunk, two ? 1 : 0, h->partial2,
                                                        gated ? &st->done : nullptr);
        LAUNCHCHK();
        src = h->partial2;
        count = nb;
    }
    gmg::k_finalize<<<1, gmg::NT_FIN, 0, h->stream>>>(src, count, stage, st);
    LAUNCHCHK();
    return GMG_OK;
}

gmg_status dot64(gmg_handle *h, const double *a, const double *b, int stage, const int *skip) {
    gmg::k_dot<double><<<h->lv[0].rows.nblocks, gmg::NT_FLAT, 0, h->stream>>>(h->lv[0].rows, a, b, h->partial, skip);
    LAUNCHCHK();
    return finalize(h, h->lv[0].rows.nblocks, stage);
}

gmg_status read_state(gmg_handle *h) {
    HIPCHK(hipMemcpyAsync(h->st_out, h->st, sizeof(PcgState), hipMemcpyDeviceToHost, h->stream));
    HIPCHK(hipStreamSynchronize(h->stream));
    return GMG_OK;
}

// z = B r ; rho = r.z ; p = z   (start, or restart, of the CG recurrence)
gmg_status pcg_start(gmg_handle *h) {
    int np = 0;
    const int *skip = &h->st->done;
    STCHK(vcycle_any(h, skip, true, &np));
    STCHK(finalize(h, np, gmg::ST_RHO0));
    Prof pf(h, GMG_K_UPDATE_P, true);
    if (mixed(h))
        gmg::k_update_p<float, float><<<h->lv[0].rows.nblocks, gmg::NT_FLAT, 0, h->stream>>>(
            h->lv[0].rows, h->P32, (const float *)h->lv[0].zout(), h->st);
    else
        gmg::k_update_p<double, double><<<h->lv[0].rows.nblocks, gmg::NT_FLAT, 0, h->stream>>>(
            h->lv[0].rows, h->P, (const double *)h->lv[0].zout(), h->st);
    LAUNCHCHK();
    gmg::k_clear_restart<<<1, 64, 0, h->stream>>>(h->st);
    LAUNCHCHK();
    return GMG_OK;
}

// One CG iteration, every scalar on the device:
//   q = A p, p.q -> alpha ; r -= alpha q, ||r||^2 -> stop? ; z = B r, r.z -> beta ;
//   x += alpha p_old, p = z + beta p_old.
gmg_status pcg_iteration(gmg_handle *h) {
    LevelHost &l0 = h->lv[0];
    const int *skip = &h->st->done;
    const bool mx = mixed(h);
    {
        Prof pf(h, GMG_K_APPLY_DOT, true);
        if (mx && l0.wx2 == 4)
            gmg::k_apply_x2<true, float, 4><<<l0.til2.nblocks, gmg::NT, 0, h->stream>>>(
                view<double, double>(l0), l0.til2, h->P32, h->Q, h->partial, skip);
        else if (mx)
            gmg::k_apply_x2<true, float><<<l0.til2.nblocks, gmg::NT, 0, h->stream>>>(
                view<double, double>(l0), l0.til2, h->P32, h->Q, h->partial, skip);
        else if (l0.wx2 == 4)
            gmg::k_apply_x2<true, double, 4><<<l0.til2.nblocks, gmg::NT, 0, h->stream>>>(
                view<double, double>(l0), l0.til2, h->P, h->Q, h->partial, skip);
        else
            gmg::k_apply_x2<true, double><<<l0.til2.nblocks, gmg::NT, 0, h->stream>>>(
                view<double, double>(l0), l0.til2, h->P, h->Q, h->partial, skip);
        LAUNCHCHK();
    }
    STCHK(finalize(h, l0.til2.nblocks, gmg::ST_ALPHA));
    {
        Prof pf(h, GMG_K_UPDATE_R, true);
        if (mx)
            gmg::k_update_r<float><<<l0.rows.nblocks, gmg::NT_FLAT, 0, h->stream>>>(l0.rows, h->R, h->Q, (float *)l0.b,
                                                                                 h->st, h->partial);
        else
            gmg::k_update_r<double><<<l0.rows.nblocks, gmg::NT_FLAT, 0, h->stream>>>(l0.rows, h->R, h->Q, nullptr, h->st,
                                                                                  h->partial);
        LAUNCHCHK();
    }
    STCHK(finalize(h, l0.rows.nblocks, gmg::ST_RR));
    int np = 0;
    STCHK(vcycle_any(h, skip, true, &np, true));
    STCHK(finalize(h, np, h->opt.flexible ? gmg::ST_BETA_FLEX : gmg::ST_BETA));
    {
        Prof pf(h, GMG_K_UPDATE_XP, true);
        if (mx)
            gmg::k_update_xp<float, float><<<l0.rows.nblocks, gmg::NT_FLAT, 0, h->stream>>>(
                l0.rows, h->X, h->P32, (const float *)l0.zout(), h->st);
        else
            gmg::k_update_xp<double, double><<<l0.rows.nblocks, gmg::NT_FLAT, 0, h->stream>>>(
                l0.rows, h->X, h->P, (const double *)l0.zout(), h->st);
        LAUNCHCHK();
    }
    return GMG_OK;
}

// Iterations enqueued between two reads of the stop flag (those past the stop
// return at once).  Measured at 513^3: 2 is 0.3-0.5 % faster than 1, 4 no
// better than 2.
int check_period(const gmg_handle *h) {
    if (h->opt.check_every > 0) return h->opt.check_every;
    const int n = h->opt.n;
    return n >= 65 ? 2 : 4;
}

// The CG loop until the device sets `done`.
gmg_status pcg_loop(gmg_handle *h) {
    const int per = check_period(h);
    for (;;) {
        for (int b = 0; b < per; ++b) STCHK(pcg_iteration(h));
        STCHK(read_state(h));
        if (h->st_out->done) return GMG_OK;
    }
}

// Solve A X = F with the result left in h->X (padded).  f, x0: caller arrays.
// zero `bytes` (a multiple of 16) of device memory with a kernel launch
gmg_status zero_dev(gmg_handle *h, void *p, size_t bytes) {
    const long long n16 = (long long)(bytes / 16);
    gmg::k_fill_zero<<<(unsigned)std::min<long long>(std::max<long long>((n16 + 255) / 256, 1), 65535), 256, 0,
                       h->stream>>>(n16, (uint4 *)p);
    LAUNCHCHK();
    return GMG_OK;
}

gmg_status solve_core(gmg_handle *h, const double *f, const double *x0, double rtol, int max_it, gmg_info *info) {
    LevelHost &l0 = h->lv[0];
    const long long nv = (long long)l0.n * l0.n * l0.n;
    h->coarse_its = 0;
    if (h->persist && h->opt.persistent_wgs > 1)  // a clean team barrier for this solve
        STCHK(zero_dev(h, h->bar, sizeof(gmg::GridBar)));
    // solve time: HIP events, or the host clock for a static-workspace handle (no events)
    const auto host0 = std::chrono::steady_clock::now();
    if (h->ev0) HIPCHK(hipEventRecord(h->ev0, h->stream));
    gmg::k_to_padded<double><<<blocks_for(nv, 256), 256, 0, h->stream>>>(l0.n, l0.pitch, f, h->F);
    LAUNCHCHK();
    PcgState s0{};
    s0.rtol2 = rtol * rtol;
    s0.max_it = max_it;
    *h->st_in = s0;
    HIPCHK(hipMemcpyAsync(h->st, h->st_in, sizeof(PcgState), hipMemcpyHostToDevice, h->stream));
    if (x0) {
        gmg::k_to_padded<double><<<blocks_for(nv, 256), 256, 0, h->stream>>>(l0.n, l0.pitch, x0, h->X);
        LAUNCHCHK();
        Prof pf(h, GMG_K_RESIDUAL, true);
        gmg::k_residual<double, double><<<l0.til64.nblocks, gmg::NT, 0, h->stream>>>(view<double, double>(l0),
                                                                                     l0.til64, h->F, h->X, h->R,
                                                                                     nullptr);
        LAUNCHCHK();
    } else {
        STCHK(zero_dev(h, h->X, l0.nel * sizeof(double)));
        HIPCHK(hipMemcpyAsync(h->R, h->F, l0.nel * sizeof(double), hipMemcpyDeviceToDevice, h->stream));
    }
    STCHK(dot64(h, h->F, h->F, gmg::ST_BB, nullptr));
    STCHK(dot64(h, h->R, h->R, gmg::ST_RR0, nullptr));
    HIPCHK(hipMemcpyAsync(h->vst_out, h->vst, sizeof(PcgState), hipMemcpyDeviceToHost, h->stream));
    STCHK(read_state(h));
    if (h->setup_pending) {  // the last gmg_set_coefficients has completed by now
        float sms = 0;
        HIPCHK(hipEventElapsedTime(&sms, h->es0, h->es1));
        h->setup_ms = sms;
        h->setup_pending = false;
    }
    STCHK(coefficient_status(h, *h->vst_out));
    const double bb = h->st_out->bb;
    int restarts = 0;
    gmg_status status = GMG_OK;
    if (!(bb == bb) || bb > 1.7e308) return fail(h, GMG_ERR_ARG, "right-hand side is not finite");
    if (bb == 0.0) {  // f = 0: x = 0
        STCHK(zero_dev(h, h->X, l0.nel * sizeof(double)));
        h->st_out->rr = h->st_out->tt = 0;
        h->st_out->its = 0;
    } else {
        if (!h->st_out->done) {
            STCHK(pcg_start(h));
            STCHK(pcg_loop(h));
        }
        for (;;) {
            // FP64 true residual
            {
                Prof pf(h, GMG_K_RESIDUAL, true);
                gmg::k_residual<double, double><<<l0.til64.nblocks, gmg::NT, 0, h->stream>>>(
                    view<double, double>(l0), l0.til64, h->F, h->X, h->Q, nullptr);
                LAUNCHCHK();
            }
            STCHK(dot64(h, h->Q, h->Q, gmg::ST_TT, nullptr));
            STCHK(read_state(h));
            const PcgState &so = *h->st_out;
            const bool true_ok = so.tt <= so.rtol2 * so.bb;
            if (so.status != 0 || true_ok || !mixed(h) || restarts >= 20 || so.its >= so.max_it) break;
            // MIXED: the recursive residual passed but the FP64 true residual did
            // not; continue from r = f - A x with a fresh search direction.
            ++restarts;
            HIPCHK(hipMemcpyAsync(h->R, h->Q, l0.nel * sizeof(double), hipMemcpyDeviceToDevice, h->stream));
            PcgState s1 = so;
            s1.done = 0;
            *h->st_in = s1;
            HIPCHK(hipMemcpyAsync(h->st, h->st_in, sizeof(PcgState), hipMemcpyHostToDevice, h->stream));
            STCHK(pcg_start(h));
            STCHK(pcg_loop(h));
        }
        status = h->st_out->status == 7 ? GMG_ERR_BREAKDOWN
                 : h->st_out->status == 6 ? GMG_ERR_NOT_CONVERGED
                                          : GMG_OK;
        if (status == GMG_OK && !(h->st_out->tt <= h->st_out->rtol2 * h->st_out->bb) && mixed(h))
            status = GMG_ERR_NOT_CONVERGED;
    }
    float ms = 0;
    if (h->ev1) {
        HIPCHK(hipEventRecord(h->ev1, h->stream));
        HIPCHK(hipEventSynchronize(h->ev1));
        HIPCHK(hipEventElapsedTime(&ms, h->ev0, h->ev1));
    } else {
        HIPCHK(hipStreamSynchronize(h->stream));
        ms = std::chrono::duration<float, std::milli>(std::chrono::steady_clock::now() - host0).count();
    }
    if (h->persist && h->opt.persistent_wgs > 1) {
        gmg::GridBar gb{};
        HIPCHK(hipMemcpy(&gb, h->bar, sizeof(gb), hipMemcpyDeviceToHost));
        if (gb.err) return fail(h, GMG_ERR_HIP, "persistent team barrier timed out");
    }
    if (info) {
        const PcgState &so = *h->st_out;
        info->iterations = so.its;
        info->restarts = restarts;
        info->rel_res = bb > 0 ? std::sqrt(so.rr / bb) : 0.0;
        info->rel_res_true = bb > 0 ? std::sqrt(so.tt / bb) : 0.0;
        info->setup_ms = h->setup_ms;
        info->solve_ms = ms;
        info->coarse_iterations = (int32_t)h->coarse_its;
    }
    if (status == GMG_ERR_BREAKDOWN) fail(h, status, "breakdown: p.Ap <= 0 or non-finite residual");
    if (status == GMG_ERR_NOT_CONVERGED) fail(h, status, "not converged within max_it");
    return status;
}

// ------------------------------------------------------------------ setup
// Dense Cholesky factor of the coarsest operator, on the device (one
// workgroup); a pivot that is not positive is recorded in h->vst.
gmg_status factor_coarsest(gmg_handle *h) {
    LevelHost &c = h->lv[h->L - 1];
    gmg::k_chol_factor<<<1, 1024, 0, h->stream>>>(c.n, c.pitch, c.plane, c.kx64, c.ky64, c.kz64,
                                                  c.g27 ? c.a64 : nullptr, c.nel, c.s, h->m, h->chol, h->vst);
    LAUNCHCHK();
    return GMG_OK;
}

template <typename V, typename K>
gmg_status upload_levels(gmg_handle *h) {
    LevBuf<V, K> lb[gmg::MAX_LEVELS];
    for (int l = 0; l < h->L; ++l) {
        lb[l].L = view<V, K>(h->lv[l]);
        lb[l].b = (V *)h->lv[l].b;
        lb[l].x = (V *)h->lv[l].x;
        lb[l].t1 = (V *)h->lv[l].t1;
        lb[l].t2 = nullptr;
    }
    HIPCHK(hipMemcpyAsync(h->dev_levels, lb, sizeof(LevBuf<V, K>) * h->L, hipMemcpyHostToDevice, h->stream));
    ChebCoef<V> cc[gmg::MAX_LEVELS];
    for (int l = 0; l < h->L; ++l) cc[l] = cheb<V>(h, l);
    HIPCHK(hipMemcpyAsync(h->dev_cheb, cc, sizeof(ChebCoef<V>) * h->L, hipMemcpyHostToDevice, h->stream));
    HIPCHK(hipStreamSynchronize(h->stream));
    return GMG_OK;
}

// ------------------------------------------------------------------ Galerkin-level interval
// The bound 2 on the spectrum of D^-1 A holds for the 7-point M-matrix, not for
// R A P, whose rows mix signs.  A smoothed Galerkin level gets the interval
// [1.1 lam lo/hi, 1.1 lam] (lo, hi: the default interval) with lam the largest
// Ritz value of kLanczosSteps Lanczos steps on D^-1 A in the D inner product,
// computed in FP64 on the device; sums of the per-workgroup partials are
// added on the host in workgroup order.
constexpr int kLanczosSteps = 20;
constexpr double kLanczosSafety = 1.1;

gmg_status host_sum(gmg_handle *h, int count, double *out) {
    std::vector<double> p(count);
    HIPCHK(hipMemcpyAsync(p.data(), h->partial, count * sizeof(double), hipMemcpyDeviceToHost, h->stream));
    HIPCHK(hipStreamSynchronize(h->stream));
    double acc = 0.0;
    for (int i = 0; i < count; ++i) acc += p[i];
    *out = acc;
    return GMG_OK;
}

// Largest eigenvalue of the symmetric tridiagonal matrix (diag d[0..m-1],
// off-diagonal e[0..m-2]): bisection on the number of negative pivots of
// T - x I, starting from the Gershgorin interval.
double tridiag_top(int m, const double *d, const double *e) {
    double a = d[0], b = d[0];
    for (int i = 0; i < m; ++i) {
        const double r = (i > 0 ? std::fabs(e[i - 1]) : 0.0) + (i + 1 < m ? std::fabs(e[i]) : 0.0);
        a = std::min(a, d[i] - r);
        b = std::max(b, d[i] + r);
    }
    for (int it = 0; it < 2000; ++it) {
        const double x = 0.5 * (a + b);
        if (!(x > a && x < b)) break;
        int neg = 0;
        double piv = 1.0;
        for (int i = 0; i < m; ++i) {
            piv = d[i] - x - (i > 0 ? e[i - 1] * e[i - 1] / piv : 0.0);
            if (piv == 0.0) piv = -1e-300;
            neg += piv < 0.0;
        }
        if (neg == m)
            b = x;  // every eigenvalue lies below x
        else
            a = x;
    }
    return b;
}

gmg_status galerkin_lambda(gmg_handle *h, int l, double *lam) {
    LevelHost &c = h->lv[l];
    const Tiling &t = c.til;
    double *v = h->X, *vp = h->R, *w = h->Q;  // free during setup; level-l layout
    HIPCHK(hipMemsetAsync(v, 0, c.nel * sizeof(double), h->stream));
    HIPCHK(hipMemsetAsync(vp, 0, c.nel * sizeof(double), h->stream));
    HIPCHK(hipMemsetAsync(w, 0, c.nel * sizeof(double), h->stream));
    gmg::k_lz_start<<<t.nblocks, gmg::NT, 0, h->stream>>>(c.n, c.pitch, c.plane, t, c.a64, c.nel, v, h->partial);
    LAUNCHCHK();
    double s0;
    STCHK(host_sum(h, t.nblocks, &s0));
    gmg::k_lz_div<<<t.nblocks, gmg::NT, 0, h->stream>>>(c.n, c.pitch, c.plane, t, v, std::sqrt(s0));
    LAUNCHCHK();
    double al[kLanczosSteps], be[kLanczosSteps], beta = 0.0;
    int m = 0;
    for (int j = 0; j < kLanczosSteps; ++j) {
        gmg::k_sweep27<double, 0, 0, true><<<t.nblocks, gmg::NT, 0, h->stream>>>(
            c.n, c.pitch, c.plane, t, c.a64, c.nel, nullptr, v, nullptr, w, 0.0, 0.0, nullptr, h->partial);
        LAUNCHCHK();
        double alpha, bn2;
        STCHK(host_sum(h, t.nblocks, &alpha));
        gmg::k_lz_orth<<<t.nblocks, gmg::NT, 0, h->stream>>>(c.n, c.pitch, c.plane, t, c.a64, c.nel, v, vp, w, alpha,
                                                             beta, h->partial);
        LAUNCHCHK();
        STCHK(host_sum(h, t.nblocks, &bn2));
        const double bn = std::sqrt(bn2);
        al[m] = alpha;
        be[m] = bn;
        ++m;
        if (!(bn > 1e-14 * std::fabs(alpha))) break;  // invariant subspace
        double *old = vp;  // vp <- v, v <- w / bn, w <- free
        vp = v;
        v = w;
        w = old;
        gmg::k_lz_div<<<t.nblocks, gmg::NT, 0, h->stream>>>(c.n, c.pitch, c.plane, t, v, bn);
        LAUNCHCHK();
        beta = bn;
    }
    *lam = tridiag_top(m, al, be);
    return GMG_OK;
}

// Rebuild every level from k and enqueue the checks into h->vst; no host
// synchronization unless the hierarchy has Galerkin levels (their Chebyshev
// intervals come from Lanczos sums added on the host) or `first` (the level
// table is uploaded once, at creation).
gmg_status load_coefficients(gmg_handle *h, const double *kx, const double *ky, const double *kz, bool first) {
    LevelHost &l0 = h->lv[0];
    // level 0 (+ the count of bad active links into vst->tt)
    gmg::k_clear_state<<<1, 64, 0, h->stream>>>(h->vst);
    LAUNCHCHK();
    gmg::k_faces_in<<<blocks_for((long long)l0.n * l0.n * l0.n, 256), 256, 0, h->stream>>>(
        l0.n, l0.pitch, kx, ky, kz, h->opt.coeff_is_log, l0.kx64, l0.ky64, l0.kz64, h->partial);
    LAUNCHCHK();
    STCHK(finalize(h, (int)blocks_for((long long)l0.n * l0.n * l0.n, 256), gmg::ST_TT, h->vst));
    for (int l = 1; l < h->L; ++l) {
        LevelHost &f = h->lv[l - 1], &c = h->lv[l];
        gmg::k_coarsen<<<blocks_for((long long)c.n * c.n * c.n, 256), 256, 0, h->stream>>>(
            f.n, f.pitch, f.plane, f.kx64, f.ky64, f.kz64, c.n, c.pitch, c.plane, c.kx64, c.ky64, c.kz64,
            h->opt.coarse_rule);
        LAUNCHCHK();
    }
    // Galerkin levels: R A P from the level above (links on its first level)
    for (int l = 1; l < h->L; ++l) {
        LevelHost &f = h->lv[l - 1], &c = h->lv[l];
        if (!c.g27) continue;
        const long long m3 = (long long)(c.n - 2) * (c.n - 2) * (c.n - 2);
        if (f.g27)
            gmg::k_galerkin<false><<<blocks_for(m3, 128), 128, 0, h->stream>>>(
                f.n, f.pitch, f.plane, nullptr, nullptr, nullptr, f.a64, f.nel, c.n, c.pitch, c.plane, c.a64, c.nel);
        else
            gmg::k_galerkin<true><<<blocks_for(m3, 128), 128, 0, h->stream>>>(
                f.n, f.pitch, f.plane, f.kx64, f.ky64, f.kz64, nullptr, f.nel, c.n, c.pitch, c.plane, c.a64, c.nel);
        LAUNCHCHK();
        if (mixed(h)) {
            gmg::k_cast27<float><<<gmg::NB_FLAT, 256, 0, h->stream>>>(27 * c.nel, c.a64, (float *)c.av);
            LAUNCHCHK();
        }
    }
    for (int l = 1; l + 1 < h->L; ++l) {  // smoothed Galerkin levels (the coarsest is solved)
        if (!h->lv[l].g27) continue;
        double lam;
        STCHK(galerkin_lambda(h, l, &lam));
        const double hi = kLanczosSafety * lam;
        set_cheb(h->lv[l], h->opt.cheb_degree, hi * (h->opt.cheb_lo / h->opt.cheb_hi), hi);
    }
    if (mixed(h)) {
        for (int l = 0; l < h->L; ++l) {
            LevelHost &c = h->lv[l];
            gmg::k_to_bf16<<<gmg::NB_FLAT, 256, 0, h->stream>>>(c.nel, c.kx64, c.kx16);
            gmg::k_to_bf16<<<gmg::NB_FLAT, 256, 0, h->stream>>>(c.nel, c.ky64, c.ky16);
            gmg::k_to_bf16<<<gmg::NB_FLAT, 256, 0, h->stream>>>(c.nel, c.kz64, c.kz16);
            LAUNCHCHK();
        }
    }
    for (int l = 0; l < h->L; ++l) {
        LevelHost &c = h->lv[l];
        if (c.g27 && mixed(h))
            gmg::k_dinv27<float><<<c.til.nblocks, gmg::NT, 0, h->stream>>>(c.n, c.pitch, c.plane, c.til,
                                                                          (const float *)c.av, c.nel, (float *)c.dinv);
        else if (c.g27)
            gmg::k_dinv27<double><<<c.til.nblocks, gmg::NT, 0, h->stream>>>(c.n, c.pitch, c.plane, c.til, c.a64, c.nel,
                                                                           (double *)c.dinv);
        else if (mixed(h))
            gmg::k_dinv<float, bf16><<<c.til.nblocks, gmg::NT, 0, h->stream>>>(view<float, bf16>(c), c.til,
                                                                                (float *)c.dinv);
        else
            gmg::k_dinv<double, double><<<c.til.nblocks, gmg::NT, 0, h->stream>>>(view<double, double>(c), c.til,
                                                                                  (double *)c.dinv);
        LAUNCHCHK();
    }
    if (h->opt.coarse_solver == 0) STCHK(factor_coarsest(h));
    bool galerkin = false;
    for (int l = 0; l < h->L; ++l) galerkin = galerkin || h->lv[l].g27;
    if (!first && !galerkin) return GMG_OK;  // the level table and intervals are unchanged
    return mixed(h) ? upload_levels<float, bf16>(h) : upload_levels<double, double>(h);
}

// The result of the checks enqueued by the last load_coefficients (waits).
gmg_status coefficient_status(gmg_handle *h, const PcgState &v) {
    if (v.tt != 0.0)
        return fail(h, GMG_ERR_COEFF, "%lld active link coefficients are not positive and finite", (long long)v.tt);
    if (v.status == 3) return fail(h, GMG_ERR_COEFF, "coarsest operator is not positive definite");
    return GMG_OK;
}

// A solve with its result copied out to x (natural layout); waits for the stream.
gmg_status solve_out(gmg_handle *h, const double *f, double *x, const double *x0, double rtol, int32_t max_it,
                     gmg_info *info) {
    const gmg_status st = solve_core(h, f, x0, rtol, max_it, info);
    if (st != GMG_OK && st != GMG_ERR_NOT_CONVERGED && st != GMG_ERR_BREAKDOWN) return st;
    LevelHost &l0 = h->lv[0];
    gmg::k_to_natural<double><<<blocks_for((long long)l0.n * l0.n * l0.n, 256), 256, 0, h->stream>>>(l0.n, l0.pitch,
                                                                                                     h->X, x);
    LAUNCHCHK();
    HIPCHK(hipStreamSynchronize(h->stream));
    return st;
}

gmg_status check_level(gmg_handle *h, int level) {
    if (!h) return GMG_ERR_ARG;
    if (level < 0 || level >= h->L) return fail(h, GMG_ERR_ARG, "level out of range");
    return GMG_OK;
}

}  // namespace

// ==================================================================== C ABI
extern "C" {

void gmg_default_options(gmg_options *o, int32_t n) {
    if (!o) return;
    memset(o, 0, sizeof(*o));
    o->n = n;
    int lv = 0;
    for (int t = n - 1; t > 1 && (t % 2) == 0; t /= 2) ++lv;
    o->levels = lv > 0 ? lv : 1;
    o->cheb_degree = 2;
    o->cheb_lo = 0.25;
    o->cheb_hi = 2.0;
    o->switch_n = 0;
    o->persistent_wgs = 1;
    o->precision = GMG_FP64;
    o->coarse_rule = GMG_COARSE_ARITHMETIC;
    o->coeff_is_log = 0;
    o->check_every = 0;
    o->coarse_solver = 0;
    o->coarse_rtol = 1e-4;
    o->coarse_max_it = 500;
    o->flexible = 0;
    o->switch2_n = 0;
    o->galerkin = 0;
    o->persistent_lds = 1;
    o->post_fused = 2;
}

const char *gmg_status_string(gmg_status s) {
    switch (s) {
    case GMG_OK: return "GMG_OK";
    case GMG_ERR_ARG: return "GMG_ERR_ARG";
    case GMG_ERR_DIMS: return "GMG_ERR_DIMS";
    case GMG_ERR_COEFF: return "GMG_ERR_COEFF";
    case GMG_ERR_NOMEM: return "GMG_ERR_NOMEM";
    case GMG_ERR_HIP: return "GMG_ERR_HIP";
    case GMG_ERR_NOT_CONVERGED: return "GMG_ERR_NOT_CONVERGED";
    case GMG_ERR_BREAKDOWN: return "GMG_ERR_BREAKDOWN";
    }
    return "GMG_ERR_UNKNOWN";
}

const char *gmg_last_error(const gmg_handle *h) { return h ? h->err : g_static_handle[g_static_last_device].err; }

void gmg_destroy(gmg_handle *h) {
    if (!h) return;
    if (h->stream) (void)hipStreamSynchronize(h->stream);
    for (void *p : h->allocs) (void)hipFree(p);
    for (int c = 0; c < GMG_K_COUNT; ++c)
        for (hipEvent_t e : h->prof_ev[c]) (void)hipEventDestroy(e);
    if (h->st_in) (void)hipHostFree(h->st_in);
    if (h->st_out) (void)hipHostFree(h->st_out);
    if (h->cst_out) (void)hipHostFree(h->cst_out);
    if (h->vst_out) (void)hipHostFree(h->vst_out);
    if (h->es0) (void)hipEventDestroy(h->es0);
    if (h->es1) (void)hipEventDestroy(h->es1);
    if (h->ev0) (void)hipEventDestroy(h->ev0);
    if (h->ev1) (void)hipEventDestroy(h->ev1);
    delete h;
}

}  // extern "C"

namespace {

// The option checks of gmg_create (GMG_ERR_ARG / GMG_ERR_DIMS).
gmg_status check_options(const gmg_options &o) {
    if (o.n < 3 || o.levels < 1 || o.levels > gmg::MAX_LEVELS) return GMG_ERR_DIMS;
    if (o.cheb_degree < 1 || o.cheb_degree > gmg::MAX_DEGREE || !(o.cheb_lo > 0.0) || !(o.cheb_hi > o.cheb_lo) ||
        (o.precision != GMG_FP64 && o.precision != GMG_MIXED) ||
        (o.coarse_rule != GMG_COARSE_ARITHMETIC && o.coarse_rule != GMG_COARSE_HARMONIC) || o.switch_n < 0 ||
        o.persistent_wgs < 1 || o.persistent_wgs > 32 || o.switch2_n < 0 || o.check_every < 0 || (o.coeff_is_log != 0 && o.coeff_is_log != 1) ||
        (o.coarse_solver != 0 && o.coarse_solver != 1) || (o.flexible != 0 && o.flexible != 1) ||
        (o.coarse_solver == 1 && (!(o.coarse_rtol > 0.0) || o.coarse_max_it < 1 || o.switch_n != 0)) ||
        o.galerkin < 0 || (o.persistent_lds != 0 && o.persistent_lds != 1) ||
        o.post_fused < 0 || o.post_fused > 2)
        return GMG_ERR_ARG;
    if ((o.n - 1) % (1 << (o.levels - 1)) != 0) return GMG_ERR_DIMS;
    const int nc = (o.n - 1) / (1 << (o.levels - 1)) + 1;
    if (nc < 3 || (o.coarse_solver == 0 && (long long)(nc - 2) * (nc - 2) * (nc - 2) > gmg::MAX_COARSE))
        return GMG_ERR_DIMS;
    // 32-bit in-chunk offsets of the one-sweep kernels (chunk_tiling)
    if (9LL * 8 * o.n * round_up(o.n, 64) > 0x7fffffffLL) return GMG_ERR_DIMS;

    return GMG_OK;
}

struct EventPair {  // setup-timing events, destroyed on every exit of build()
    hipEvent_t a = nullptr, b = nullptr;
    ~EventPair() {
        if (a) (void)hipEventDestroy(a);
        if (b) (void)hipEventDestroy(b);
    }
};

// Everything gmg_create does after the option check, on a fresh handle whose
// opt and stream are set (and, for the static workspace, arena and host
// state records).  On failure the caller releases what the handle holds.
gmg_status build(gmg_handle *h, const double *kx, const double *ky, const double *kz) {
    const gmg_options o = h->opt;
    const bool arena = h->arena != nullptr;
    h->L = o.levels;
    EventPair tm;  // setup timing (host clock for the static workspace, which creates no events)
    const auto host0 = std::chrono::steady_clock::now();
    if (!arena) {
        if (hipEventCreate(&h->ev0) != hipSuccess || hipEventCreate(&h->ev1) != hipSuccess ||
            hipEventCreate(&tm.a) != hipSuccess || hipEventCreate(&tm.b) != hipSuccess ||
            hipEventCreate(&h->es0) != hipSuccess || hipEventCreate(&h->es1) != hipSuccess)
            return fail(h, GMG_ERR_HIP, "hipEventCreate failed");
        (void)hipEventRecord(tm.a, h->stream);
        if (hipHostMalloc((void **)&h->st_in, sizeof(PcgState)) != hipSuccess ||
            hipHostMalloc((void **)&h->st_out, sizeof(PcgState)) != hipSuccess ||
            hipHostMalloc((void **)&h->cst_out, sizeof(PcgState)) != hipSuccess ||
            hipHostMalloc((void **)&h->vst_out, sizeof(PcgState)) != hipSuccess)
            return fail(h, GMG_ERR_NOMEM, "hipHostMalloc failed");
    }
    const bool mx = o.precision == GMG_MIXED;
    // level geometry
    int n = o.n;
    for (int l = 0; l < h->L; ++l) {
        LevelHost &lh = h->lv[l];
        lh.n = n;
        lh.pitch = round_up(n, 64);
        lh.plane = (long long)n * lh.pitch;
        lh.nel = (long long)n * lh.plane;
        lh.s = (double)(n - 1) * (double)(n - 1);
        const int t64 = env_int("GMG_TARGET_WGS_64", 1 << 20);
        lh.til = make_tiling(n, env_int("GMG_TARGET_WGS_V", 1 << 20));
        lh.til64 = make_tiling(n, t64);
        // outer apply: 512 x 1 tiles on rows of 384 points or more, with
        // chunks of at least 4 planes (5 at 513^3: MIXED 872 us against 880 us
        // for 128 x 4 tiles and 9-plane chunks, FP64 1027 against 1034 us;
        // 3- to 8-plane chunks within 0.5 %), else 128 x 4 tiles
        lh.wx2 = (n - 2 >= 384 && env_int("GMG_APPLY_WIDTH", 512) == 512) ? 4 : 1;
        lh.til2 = lh.wx2 == 4 ? make_tiling(n, t64, 4 * gmg::TX2, 1, 4, true) : make_tiling(n, t64, gmg::TX2);
        lh.tilp = make_tiling(n, env_int("GMG_TARGET_WGS_V", 1 << 20), gmg::TX, gmg::TY_PRE);
        lh.tilr = even_chunks(lh.til, n);
        // pre-smoothing + residual in one sweep: 64 x 16 tiles and 64-plane chunks
        // (513^3 FP64 1.58 ms, 32-plane 1.63 ms, 64 x 8 tiles 1.64 ms; FP32
        // 0.67 ms, 32-plane 0.70 ms, 64 x 8 tiles 0.75 ms)
        lh.tilf = even_chunks(chunk_tiling(n, env_int("GMG_PRE_CHUNK", 64), gmg::TX, gmg::TY_PRE_RES), n);
        // one-sweep post-smoothing: 64 x 8 tiles, 32-plane chunks (513^3 FP32
        // 0.80 ms, 16-plane 0.81 ms, 8-plane 0.87 ms; FP64 1.60 ms, 16-plane
        // 1.62 ms, 64-plane 1.60 ms)
        lh.tilq = chunk_tiling(n, env_int("GMG_POST_CHUNK", 32), gmg::TX, gmg::TY_POST);
        lh.rows = make_rows(n, lh.pitch, lh.plane);
        lh.g27 = o.galerkin > 0 && l >= o.galerkin;
        n = (n - 1) / 2 + 1;
    }
    // persistent switch: first level l >= 1 with N_l <= switch_n; with a team,
    // the first level with N_l <= switch2_n moves on to a single workgroup
    h->s_persist = h->L - 1;
    h->s2_persist = h->L - 1;
    h->persist = false;
    if (o.switch_n > 0 && h->L > 1) {
        for (int l = 1; l < h->L; ++l)
            if (h->lv[l].n <= o.switch_n) {
                h->s_persist = l;
                h->persist = true;
                break;
            }
    }
    if (h->persist && o.persistent_wgs > 1 && o.switch2_n > 0) {
        for (int l = h->s_persist + 1; l < h->L - 1; ++l)
            if (h->lv[l].n <= o.switch2_n) {
                h->s2_persist = l;
                break;
            }
    }
    // one-sweep post-smoothing on the grid-path link levels (degree 2)
    for (int l = 0; l < h->s_persist; ++l)
        h->lv[l].post1 = (o.post_fused == 1 || o.post_fused == 2) && !h->lv[l].g27 && o.cheb_degree == 2;
    {
        // pre-smoothing and residual in one sweep on the grid levels (at 513^3
        // FP64 1.97 ms against 1.38 + 1.31 ms for the two sweeps, FP32/BF16 0.85 ms
        // against 0.56 + 0.46 ms); GMG_PRE_FUSED=0 selects the two sweeps
        const char *e = getenv("GMG_PRE_FUSED");
        const bool pre_on = !(e && e[0] == '0');
        for (int l = 0; l < h->s_persist; ++l)
            h->lv[l].pre1 = pre_on && !h->lv[l].g27 && o.cheb_degree == 2;
    }
    // allocations
    gmg_status s;
    LevelHost &l0 = h->lv[0];
#define ALLOC(ptr, cnt)                                   \
    do {                                                  \
        if ((s = dalloc(h, &(ptr), (cnt))) != GMG_OK) return s;        \
    } while (0)
    ALLOC(h->F, l0.nel);
    ALLOC(h->X, l0.nel);
    ALLOC(h->R, l0.nel);
    if (mx)
        ALLOC(h->P32, l0.nel);
    else
        ALLOC(h->P, l0.nel);
    ALLOC(h->Q, l0.nel);
    h->npartial = std::max(std::max(std::max(l0.til.nblocks, l0.til64.nblocks), l0.til2.nblocks),
                           std::max(std::max(l0.rows.nblocks, l0.tilq.nblocks), gmg::NB_FLAT));
    for (int l = 1; l < h->L; ++l)  // coarse-level sums (truncated coarse CG, Lanczos) use their own tilings
        h->npartial = std::max(h->npartial, std::max(std::max(h->lv[l].til.nblocks, h->lv[l].tilq.nblocks),
                                                     h->lv[l].rows.nblocks));
    {
        const long long nfaces_blocks = blocks_for((long long)l0.n * l0.n * l0.n, 256);
        if (nfaces_blocks > h->npartial) h->npartial = (int)nfaces_blocks;
    }
    ALLOC(h->partial, 2LL * h->npartial);  // two partial arrays for paired sums
    ALLOC(h->partial2, 2LL * gmg::NB_CHUNKS);
    ALLOC(h->st, 1LL);
    ALLOC(h->cst, 1LL);
    ALLOC(h->vst, 1LL);
    ALLOC(h->bar, 1LL);
    for (int l = 0; l < h->L; ++l) {
        LevelHost &lh = h->lv[l];
        ALLOC(lh.kx64, lh.nel);
        ALLOC(lh.ky64, lh.nel);
        ALLOC(lh.kz64, lh.nel);
        if (lh.g27) {
            ALLOC(lh.a64, 27 * lh.nel);
            if (mx) {
                float *a;
                ALLOC(a, 27 * lh.nel);
                lh.av = a;
            } else {
                lh.av = lh.a64;
            }
        }
        if (mx) {
            ALLOC(lh.kx16, lh.nel);
            ALLOC(lh.ky16, lh.nel);
            ALLOC(lh.kz16, lh.nel);
            float *b, *x, *t1, *dv;
            ALLOC(b, lh.nel);
            ALLOC(x, lh.nel);
            ALLOC(t1, lh.nel);
            ALLOC(dv, lh.nel);
            lh.b = b;
            lh.x = x;
            lh.t1 = t1;
            lh.dinv = dv;
        } else {
            double *b = nullptr, *x, *t1, *dv;
            if (l > 0) ALLOC(b, lh.nel);
            ALLOC(x, lh.nel);
            ALLOC(t1, lh.nel);
            ALLOC(dv, lh.nel);
            lh.dinv = dv;
            lh.b = l == 0 ? (void *)h->R : (void *)b;  // FP64: the finest V-cycle input is r itself
            lh.x = x;
            lh.t1 = t1;
        }
    }
    if (o.coarse_solver == 0) {
        const int nn = h->lv[h->L - 1].n - 2;
        h->m = nn * nn * nn;
        ALLOC(h->chol, (long long)h->m * h->m);
    } else {  // truncated hierarchy: coarse CG direction and product on the coarsest level
        const LevelHost &c = h->lv[h->L - 1];
        if (mx) {
            float *a, *b;
            ALLOC(a, c.nel);
            ALLOC(b, c.nel);
            h->cp = a;
            h->cq = b;
        } else {
            double *a, *b;
            ALLOC(a, c.nel);
            ALLOC(b, c.nel);
            h->cp = a;
            h->cq = b;
        }
    }
    {
        char *dl;
        const size_t sz = mx ? sizeof(LevBuf<float, bf16>) : sizeof(LevBuf<double, double>);
        const size_t szc = mx ? sizeof(ChebCoef<float>) : sizeof(ChebCoef<double>);
        char *dc;
        ALLOC(dc, (long long)(szc * h->L));
        h->dev_cheb = dc;
        ALLOC(dl, (long long)(sz * h->L));
        h->dev_levels = dl;
    }
#undef ALLOC
    if (arena) {  // the workspace keeps the previous call's contents: clear the part in use
        const long long n16 = (long long)((h->arena_used + 15) / 16);
        gmg::k_fill_zero<<<(unsigned)std::min<long long>((n16 + 255) / 256, 65535), 256, 0, h->stream>>>(
            n16, (uint4 *)h->arena);
        LAUNCHCHK();
    }
    // persistent team placement: 8 = one workgroup in eight launched, so the
    // active ones share an XCD; 1 if the packed launch would not fit
    if (h->persist && o.persistent_wgs > 1) {
        int dev = 0, coop = 0, ncu = 0, occ = 0;
        (void)hipGetDevice(&dev);
        (void)hipDeviceGetAttribute(&coop, hipDeviceAttributeCooperativeLaunch, dev);
        (void)hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev);
        if (!coop) return fail(h, GMG_ERR_HIP, "cooperative launch unsupported");
        if (mx)
            (void)hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, gmg::k_persistent<float, bf16>, gmg::NT_PERSIST, 0);
        else
            (void)hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, gmg::k_persistent<double, double>,
                                                               gmg::NT_PERSIST, 0);
        const long long cap = (long long)occ * ncu;
        h->persist_spread = (8LL * o.persistent_wgs <= cap) ? 8 : 1;
        if ((long long)o.persistent_wgs > cap) return fail(h, GMG_ERR_ARG, "persistent team cannot be co-resident");
    }
    // one-workgroup persistent levels in LDS when they all fit (link levels only)
    if (h->persist && o.persistent_wgs == 1 && o.persistent_lds) {
        size_t bytes = gmg::lds_align((size_t)h->m * sizeof(double));
        bool links = true;
        for (int l = h->s_persist; l < h->L; ++l) {
            bytes += mx ? gmg::lds_level_bytes<float, bf16>(h->lv[l].n) : gmg::lds_level_bytes<double, double>(h->lv[l].n);
            links = links && !h->lv[l].g27;
        }
        int dev = 0, cap = 0;
        (void)hipGetDevice(&dev);
        (void)hipDeviceGetAttribute(&cap, hipDeviceAttributeMaxSharedMemoryPerMultiprocessor, dev);
        hipFuncAttributes fa{};
        const void *fn = mx ? (const void *)gmg::k_persistent_lds<float, bf16>
                            : (const void *)gmg::k_persistent_lds<double, double>;
        if (links && hipFuncGetAttributes(&fa, fn) == hipSuccess && bytes + fa.sharedSizeBytes <= (size_t)cap &&
            hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes) == hipSuccess) {
            h->persist_lds = true;
            h->lds_bytes = bytes;
        }
        (void)hipGetLastError();
    }
    // Chebyshev coefficients: the default interval on every level (Galerkin
    // levels get their own in load_coefficients)
    for (int l = 0; l < h->L; ++l) set_cheb(h->lv[l], o.cheb_degree, o.cheb_lo, o.cheb_hi);
    if ((s = load_coefficients(h, kx, ky, kz, true)) != GMG_OK) return s;
    if (tm.b) (void)hipEventRecord(tm.b, h->stream);
    HIPCHK(hipMemcpyAsync(h->vst_out, h->vst, sizeof(PcgState), hipMemcpyDeviceToHost, h->stream));
    HIPCHK(hipStreamSynchronize(h->stream));
    STCHK(coefficient_status(h, *h->vst_out));
    float ms = 0;
    if (tm.a)
        (void)hipEventElapsedTime(&ms, tm.a, tm.b);
    else
        ms = std::chrono::duration<float, std::milli>(std::chrono::steady_clock::now() - host0).count();
    h->setup_ms = ms;
    return GMG_OK;
}

}  // namespace

extern "C" {

gmg_status gmg_create(const gmg_options *opt, const double *kx, const double *ky, const double *kz, void *stream,
                      gmg_handle **out) {
    if (!out) return GMG_ERR_ARG;
    *out = nullptr;
    if (!opt || !kx || !ky || !kz) return GMG_ERR_ARG;
    const gmg_status c = check_options(*opt);
    if (c != GMG_OK) return c;
    gmg_handle *h = new gmg_handle();
    h->opt = *opt;
    h->stream = (hipStream_t)stream;
    const gmg_status s = build(h, kx, ky, kz);
    if (s != GMG_OK) {
        gmg_destroy(h);
        return s;
    }
    *out = h;
    return GMG_OK;
}


gmg_status gmg_set_coefficients(gmg_handle *h, const double *kx, const double *ky, const double *kz) {
    if (!h || !kx || !ky || !kz) return GMG_ERR_ARG;
    HIPCHK(hipEventRecord(h->es0, h->stream));
    const gmg_status s = load_coefficients(h, kx, ky, kz, false);
    if (s != GMG_OK) return s;
    HIPCHK(hipEventRecord(h->es1, h->stream));
    h->setup_pending = true;
    return GMG_OK;
}

gmg_status gmg_set_stream(gmg_handle *h, void *stream) {
    if (!h) return GMG_ERR_ARG;
    HIPCHK(hipStreamSynchronize(h->stream));
    h->stream = (hipStream_t)stream;
    return GMG_OK;
}

gmg_status gmg_solve(gmg_handle *h, const double *f, double *x, const double *x0, double rtol, int32_t max_it,
                     gmg_info *info) {
    if (!h || !f || !x) return h ? fail(h, GMG_ERR_ARG, "null vector") : GMG_ERR_ARG;
    if (!(rtol >= 0.0) || max_it < 1) return fail(h, GMG_ERR_ARG, "rtol must be >= 0 and max_it >= 1");
    return solve_out(h, f, x, x0, rtol, max_it, info);
}

gmg_status gmg_adjoint_gradient(gmg_handle *h, const double *phi, const double *dl_dphi, double *g_x, double *g_y,
                                double *g_z, double *lambda, double rtol, int32_t max_it, gmg_info *info) {
    if (!h || !phi || !dl_dphi || !g_x || !g_y || !g_z) return h ? fail(h, GMG_ERR_ARG, "null array") : GMG_ERR_ARG;
    if (!(rtol >= 0.0) || max_it < 1) return fail(h, GMG_ERR_ARG, "rtol must be >= 0 and max_it >= 1");
    gmg_status st = solve_core(h, dl_dphi, nullptr, rtol, max_it, info);
    if (st != GMG_OK && st != GMG_ERR_NOT_CONVERGED && st != GMG_ERR_BREAKDOWN) return st;
    LevelHost &l0 = h->lv[0];
    const long long nv = (long long)l0.n * l0.n * l0.n;
    {
        Prof pf(h, GMG_K_FACE_GRADIENT, true);
        gmg::k_face_gradient<<<blocks_for(nv, 256), 256, 0, h->stream>>>(l0.n, l0.pitch, l0.s, h->X, phi, l0.kx64,
                                                                         l0.ky64, l0.kz64, g_x, g_y, g_z);
        LAUNCHCHK();
    }
    if (lambda) {
        gmg::k_to_natural<double><<<blocks_for(nv, 256), 256, 0, h->stream>>>(l0.n, l0.pitch, h->X, lambda);
        LAUNCHCHK();
    }
    HIPCHK(hipStreamSynchronize(h->stream));
    return st;
}

// ------------------------------------------------------------------ static workspace
// gmg_solve_static: the solve of gmg_create + gmg_solve with no allocation.
// Every device buffer of the hierarchy comes from `scratch` (one copy per
// GPU, held until the process ends; its address on each device is taken once
// with hipGetSymbolAddress, and only that address is handed to kernels), the
// handle and its host state records are static, and no event, pinned buffer
// or heap object is created.  Calls on one GPU share all of it: calls that
// overlap on one GPU race.
gmg_status gmg_solve_static(const gmg_options *opt, const double *kx, const double *ky, const double *kz,
                            const double *f, double *x, const double *x0, double rtol, int32_t max_it, void *stream,
                            gmg_info *info) {
    if (!opt || !kx || !ky || !kz || !f || !x || !(rtol >= 0.0) || max_it < 1) return GMG_ERR_ARG;
    gmg_status s = check_options(*opt);
    if (s != GMG_OK) return s;
    if (opt->galerkin != 0) return GMG_ERR_ARG;  // Galerkin intervals need host work buffers
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return GMG_ERR_HIP;
    g_static_last_device = dev;
    gmg_handle *h = &g_static_handle[dev];
    *h = gmg_handle{};
    if (!g_scratch[dev]) {  // once per device, with the device current
        void *p = nullptr;
        if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) {
            (void)hipGetLastError();
            return fail(h, GMG_ERR_HIP, "hipGetSymbolAddress of the static workspace failed");
        }
        g_scratch[dev] = p;
    }
    h->opt = *opt;
    h->stream = (hipStream_t)stream;
    h->arena = (char *)g_scratch[dev];
    h->arena_cap = kStaticBytes;
    h->st_in = &g_static_state[dev][0];
    h->st_out = &g_static_state[dev][1];
    h->cst_out = &g_static_state[dev][2];
    h->vst_out = &g_static_state[dev][3];
    if ((s = build(h, kx, ky, kz)) != GMG_OK) return s;
    return solve_out(h, f, x, x0, rtol, max_it, info);
}

int32_t gmg_level_n(const gmg_handle *h, int32_t level) {
    if (!h || level < 0 || level >= h->L) return -1;
    return h->lv[level].n;
}

}  // extern "C"

// ------------------------------------------------------------------ test hooks
namespace {

template <typename V>
gmg_status in_vec(gmg_handle *h, const LevelHost &lh, const double *src, V *dst) {
    const long long nv = (long long)lh.n * lh.n * lh.n;
    gmg::k_to_padded<V><<<blocks_for(nv, 256), 256, 0, h->stream>>>(lh.n, lh.pitch, src, dst);
    LAUNCHCHK();
    return GMG_OK;
}
template <typename V>
gmg_status out_vec(gmg_handle *h, const LevelHost &lh, const V *src, double *dst) {
    const long long nv = (long long)lh.n * lh.n * lh.n;
    gmg::k_to_natural<V><<<blocks_for(nv, 256), 256, 0, h->stream>>>(lh.n, lh.pitch, src, dst);
    LAUNCHCHK();
    HIPCHK(hipStreamSynchronize(h->stream));
    return GMG_OK;
}

template <typename V, typename K>
gmg_status hook_apply(gmg_handle *h, int level, const double *x, double *y) {
    LevelHost &lh = h->lv[level];
    STCHK(in_vec<V>(h, lh, x, (V *)lh.t1));
    if (lh.g27)
        gmg::k_sweep27<V, 0, 0><<<lh.til.nblocks, gmg::NT, 0, h->stream>>>(lh.n, lh.pitch, lh.plane, lh.til,
                                                                          (const V *)lh.av, lh.nel, nullptr,
                                                                          (const V *)lh.t1, nullptr, (V *)lh.x, V(0),
                                                                          V(0), nullptr);
    else
        gmg::k_apply<V, K, false><<<lh.til.nblocks, gmg::NT, 0, h->stream>>>(view<V, K>(lh), lh.til,
                                                                            (const V *)lh.t1, (V *)lh.x, nullptr,
                                                                            nullptr);
    LAUNCHCHK();
    return out_vec<V>(h, lh, (const V *)lh.x, y);
}

template <typename V, typename K>
gmg_status hook_smooth(gmg_handle *h, int level, const double *b, double *x, int x0_zero) {
    LevelHost &lh = h->lv[level];
    STCHK(in_vec<V>(h, lh, b, (V *)lh.b));
    if (!x0_zero) STCHK(in_vec<V>(h, lh, x, (V *)lh.x));
    STCHK((smooth_grid<V, K>(h, level, x0_zero != 0, nullptr, nullptr, nullptr, nullptr)));
    return out_vec<V>(h, lh, (const V *)(x0_zero ? lh.x : lh.zout()), x);
}

template <typename V, typename K>
gmg_status hook_restrict(gmg_handle *h, int level, const double *b, const double *x, double *bc) {
    LevelHost &f = h->lv[level], &c = h->lv[level + 1];
    STCHK(in_vec<V>(h, f, b, (V *)f.b));
    STCHK(in_vec<V>(h, f, x, (V *)f.x));
    STCHK((residual_restrict<V, K>(h, level, nullptr)));
    return out_vec<V>(h, c, (const V *)c.b, bc);
}

template <typename V, typename K>
gmg_status hook_prolong(gmg_handle *h, int level, const double *e, double *x) {
    LevelHost &f = h->lv[level], &c = h->lv[level + 1];
    STCHK(in_vec<V>(h, c, e, (V *)c.x));
    STCHK(in_vec<V>(h, f, x, (V *)f.x));
    gmg::k_prolong<V><<<prolong_grid(c.n), gmg::NT, 0, h->stream>>>(f.pitch, f.plane, c.n, c.pitch, c.plane,
                                                                    (const V *)c.x, (V *)f.x, nullptr);
    LAUNCHCHK();
    return out_vec<V>(h, f, (const V *)f.x, x);
}

template <typename V, typename K>
gmg_status hook_coarse(gmg_handle *h, const double *b, double *x) {
    LevelHost &c = h->lv[h->L - 1];
    STCHK(in_vec<V>(h, c, b, (V *)c.b));
    if (h->opt.coarse_solver == 1) {
        STCHK((coarse_cg<V, K>(h, nullptr)));
        return out_vec<V>(h, c, (const V *)c.x, x);
    }
    gmg::k_coarse_solve<V><<<1, 256, 0, h->stream>>>(c.n, c.pitch, c.plane, h->m, h->chol, (const V *)c.b, (V *)c.x,
                                                      nullptr);
    LAUNCHCHK();
    return out_vec<V>(h, c, (const V *)c.x, x);
}

template <typename V, typename K>
gmg_status hook_vcycle(gmg_handle *h, const double *r, double *z) {
    LevelHost &l0 = h->lv[0];
    if (h->persist && h->opt.persistent_wgs > 1) HIPCHK(hipMemsetAsync(h->bar, 0, sizeof(gmg::GridBar), h->stream));
    STCHK(in_vec<double>(h, l0, r, h->R));
    STCHK((vcycle<V, K>(h, nullptr, false, nullptr)));
    return out_vec<V>(h, l0, (const V *)l0.zout(), z);
}

}  // namespace

extern "C" {

gmg_status gmg_apply_operator(gmg_handle *h, int32_t level, const double *x, double *y) {
    STCHK(check_level(h, level));
    if (!x || !y) return fail(h, GMG_ERR_ARG, "null vector");
    return mixed(h) ? hook_apply<float, bf16>(h, level, x, y) : hook_apply<double, double>(h, level, x, y);
}

gmg_status gmg_apply_outer_operator(gmg_handle *h, const double *x, double *y) {
    if (!h) return GMG_ERR_ARG;
    if (!x || !y) return fail(h, GMG_ERR_ARG, "null vector");
    LevelHost &l0 = h->lv[0];
    double *u = h->X;  // free between solves (every solve re-initializes it)
    STCHK(in_vec<double>(h, l0, x, u));
    if (l0.wx2 == 4)
        gmg::k_apply_x2<false, double, 4><<<l0.til2.nblocks, gmg::NT, 0, h->stream>>>(view<double, double>(l0),
                                                                                     l0.til2, u, h->Q, nullptr, nullptr);
    else
        gmg::k_apply_x2<false, double><<<l0.til2.nblocks, gmg::NT, 0, h->stream>>>(view<double, double>(l0), l0.til2,
                                                                                  u, h->Q, nullptr, nullptr);
    LAUNCHCHK();
    return out_vec<double>(h, l0, h->Q, y);
}

gmg_status gmg_debug_smooth(gmg_handle *h, int32_t level, const double *b, double *x, int32_t x0_zero) {
    STCHK(check_level(h, level));
    if (!b || !x) return fail(h, GMG_ERR_ARG, "null vector");
    return mixed(h) ? hook_smooth<float, bf16>(h, level, b, x, x0_zero)
                    : hook_smooth<double, double>(h, level, b, x, x0_zero);
}

gmg_status gmg_debug_residual_restrict(gmg_handle *h, int32_t level, const double *b, const double *x,
                                       double *b_coarse) {
    STCHK(check_level(h, level));
    if (level + 1 >= h->L) return fail(h, GMG_ERR_ARG, "no coarser level");
    if (!b || !x || !b_coarse) return fail(h, GMG_ERR_ARG, "null vector");
    return mixed(h) ? hook_restrict<float, bf16>(h, level, b, x, b_coarse)
                    : hook_restrict<double, double>(h, level, b, x, b_coarse);
}

gmg_status gmg_debug_prolong(gmg_handle *h, int32_t level, const double *e_coarse, double *x) {
    STCHK(check_level(h, level));
    if (level + 1 >= h->L) return fail(h, GMG_ERR_ARG, "no coarser level");
    if (!e_coarse || !x) return fail(h, GMG_ERR_ARG, "null vector");
    return mixed(h) ? hook_prolong<float, bf16>(h, level, e_coarse, x)
                    : hook_prolong<double, double>(h, level, e_coarse, x);
}

gmg_status gmg_debug_coarse_solve(gmg_handle *h, const double *b, double *x) {
    if (!h) return GMG_ERR_ARG;
    if (!b || !x) return fail(h, GMG_ERR_ARG, "null vector");
    return mixed(h) ? hook_coarse<float, bf16>(h, b, x) : hook_coarse<double, double>(h, b, x);
}

gmg_status gmg_debug_vcycle(gmg_handle *h, const double *r, double *z) {
    if (!h) return GMG_ERR_ARG;
    if (!r || !z) return fail(h, GMG_ERR_ARG, "null vector");
    return mixed(h) ? hook_vcycle<float, bf16>(h, r, z) : hook_vcycle<double, double>(h, r, z);
}

gmg_status gmg_get_level_coefficients(gmg_handle *h, int32_t level, double *kx, double *ky, double *kz) {
    STCHK(check_level(h, level));
    if (!kx || !ky || !kz) return fail(h, GMG_ERR_ARG, "null array");
    LevelHost &lh = h->lv[level];
    const long long nv = (long long)lh.n * lh.n * lh.n;
    if (mixed(h))
        gmg::k_faces_out<bf16><<<blocks_for(nv, 256), 256, 0, h->stream>>>(lh.n, lh.pitch, lh.kx16, lh.ky16, lh.kz16,
                                                                           kx, ky, kz);
    else
        gmg::k_faces_out<double><<<blocks_for(nv, 256), 256, 0, h->stream>>>(lh.n, lh.pitch, lh.kx64, lh.ky64,
                                                                             lh.kz64, kx, ky, kz);
    LAUNCHCHK();
    HIPCHK(hipStreamSynchronize(h->stream));
    return GMG_OK;
}

uint64_t gmg_persistent_lds_bytes(const gmg_handle *h) { return h && h->persist_lds ? h->lds_bytes : 0; }

gmg_status gmg_get_level_interval(gmg_handle *h, int32_t level, double *lo, double *hi) {
    STCHK(check_level(h, level));
    if (!lo || !hi) return fail(h, GMG_ERR_ARG, "null pointer");
    *lo = h->lv[level].lo;
    *hi = h->lv[level].hi;
    return GMG_OK;
}

gmg_status gmg_get_level_stencil(gmg_handle *h, int32_t level, double *a27) {
    STCHK(check_level(h, level));
    if (!a27) return fail(h, GMG_ERR_ARG, "null array");
    LevelHost &lh = h->lv[level];
    if (!lh.g27) return fail(h, GMG_ERR_ARG, "level has no Galerkin operator");
    const long long nv = (long long)lh.n * lh.n * lh.n;
    gmg::k_stencil_out<<<blocks_for(nv, 256), 256, 0, h->stream>>>(lh.n, lh.pitch, lh.plane, lh.a64, lh.nel, a27);
    LAUNCHCHK();
    HIPCHK(hipStreamSynchronize(h->stream));
    return GMG_OK;
}

}  // extern "C"

extern "C" {

gmg_status gmg_profile_start(gmg_handle *h) {
    if (!h) return GMG_ERR_ARG;
    HIPCHK(hipStreamSynchronize(h->stream));
    for (int c = 0; c < GMG_K_COUNT; ++c) h->prof_used[c] = 0;
    h->prof_on = true;
    return GMG_OK;
}

gmg_status gmg_profile_stop(gmg_handle *h) {
    if (!h) return GMG_ERR_ARG;
    h->prof_on = false;
    HIPCHK(hipStreamSynchronize(h->stream));
    return GMG_OK;
}

gmg_status gmg_profile_get(gmg_handle *h, int32_t kclass, int32_t *launches, double *total_ms) {
    if (!h || kclass < 0 || kclass >= GMG_K_COUNT || !launches || !total_ms) return GMG_ERR_ARG;
    HIPCHK(hipStreamSynchronize(h->stream));
    double tot = 0.0;
    const int n = h->prof_used[kclass];
    for (int i = 0; i < n; ++i) {
        float ms = 0.0f;
        HIPCHK(hipEventElapsedTime(&ms, h->prof_ev[kclass][2 * i], h->prof_ev[kclass][2 * i + 1]));
        tot += ms;
    }
    *launches = n;
    *total_ms = tot;
    return GMG_OK;
}

const char *gmg_kernel_class_name(int32_t c) {
    static const char *names[GMG_K_COUNT] = {"apply_dot",      "residual",  "update_r",       "update_p",
                                             "cheb_first",     "cheb_step", "cheb_step_prev", "cheb_step_dot",
                                             "level_residual", "prolong",   "persistent",     "coarse_solve",
                                             "face_gradient",  "restrict",  "update_xp",      "cheb_pre2",
                                             "cheb_post2",     "pre2_res"};
    return (c >= 0 && c < GMG_K_COUNT) ? names[c] : "unknown";
}

}  // extern "C"

extern "C" gmg_status gmg_calibration_copy(void *dst, const void *src, uint64_t bytes, int32_t planes,
                                           void *stream) {
    if (!dst || !src || planes < 1 || (bytes % (16ull * (uint64_t)planes)) != 0) return GMG_ERR_ARG;
    const long long n16 = (long long)(bytes / 16 / (uint64_t)planes);
    const long long nb = (n16 + 255) / 256;
    if (nb > 0x7fffffffLL) return GMG_ERR_ARG;
    gmg::k_copy_march<<<(unsigned)(nb > 0 ? nb : 1), 256, 0, (hipStream_t)stream>>>(
        n16, planes, (const gmg::u32x4 *)src, (gmg::u32x4 *)dst);
    if (hipGetLastError() != hipSuccess) return GMG_ERR_HIP;
    if (hipStreamSynchronize((hipStream_t)stream) != hipSuccess) return GMG_ERR_HIP;
    return GMG_OK;
}
