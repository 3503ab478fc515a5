// kernels.hpp -- HIP device code (gfx950) for the multigrid-preconditioned CG
// solve of -div(k grad phi) = f on a structured 3D vertex grid.
//
// Storage used by every kernel (one "level"):
//   * vertex (i,j,k) of an N^3 grid lives at element  k*plane + j*pitch + i,
//     pitch = N rounded up to a multiple of 64 elements, plane = N*pitch, so
//     every row starts on a 128-byte boundary for FP64, FP32 and BF16 alike;
//   * kx[o] is the coefficient of the link (i,j,k)-(i+1,j,k) stored at the
//     offset o of its lower end point (ky, kz likewise along y, z);
//   * boundary vertices and padding hold 0 in every vector and are never
//     written, so vector kernels may sweep whole rows including them.
//
// Two precisions share the code through templates: V is the arithmetic /
// vector type (double or float) and K the stored coefficient type (double or
// bfloat16 bits).  Arithmetic is written with explicit fused multiply-adds and
// the file is compiled with -ffp-contract=off, so every code path that calls the
// same value function (grid kernels, the persistent coarse kernel) rounds
// identically.
#pragma once
#include <hip/hip_runtime.h>
#include <type_traits>
#include <stdint.h>

namespace gmg {

typedef uint16_t bf16;

constexpr int TX = 64;          // threads along x in a stencil tile (one wave64 row)
constexpr int TY = 4;           // rows per tile
constexpr int NT = TX * TY;     // threads per stencil workgroup
constexpr int TX2 = 2 * TX;     // x extent of a tile of the two-points-per-lane apply
constexpr int TY_PRE = 2 * TY;  // rows per tile of the two-rows-per-thread pre-smoothing kernel
constexpr int TY_POST = 8;      // rows per tile of the one-sweep post-smoothing kernel
constexpr int TY_PRE_RES = 16;  // rows per tile of the one-sweep pre-smoothing + residual kernel
constexpr int NT_FLAT = 256;    // threads per workgroup of the flat vector kernels
constexpr int NB_FLAT = 2048;   // workgroups of the flat vector kernels (fixed => deterministic sums)
constexpr int NT_PERSIST = 1024;
constexpr int MAX_LEVELS = 16;
constexpr int MAX_DEGREE = 8;
constexpr int MAX_COARSE = 4096;  // interior unknowns of the coarsest level (dense Cholesky)

// ---------------------------------------------------------------- scalars
__device__ __forceinline__ double fmaT(double a, double b, double c) { return __fma_rn(a, b, c); }
__device__ __forceinline__ float fmaT(float a, float b, float c) { return __fmaf_rn(a, b, c); }
__device__ __forceinline__ double kval(double v) { return v; }
__device__ __forceinline__ float kval(bf16 v) { return __uint_as_float(((uint32_t)v) << 16); }
// Streaming (nontemporal) loads and stores for data a kernel touches once.
template <typename T>
__device__ __forceinline__ T ldnt(const T *p) { return __builtin_nontemporal_load(p); }
template <typename T>
__device__ __forceinline__ void stnt(T v, T *p) { __builtin_nontemporal_store(v, p); }
// Pair forms: one 8- or 16-byte access (the address must be aligned to its size).
typedef float f32x2 __attribute__((ext_vector_type(2)));
typedef double f64x2 __attribute__((ext_vector_type(2)));
__device__ __forceinline__ float2 ldnt(const float2 *p) {
    const f32x2 v = __builtin_nontemporal_load((const f32x2 *)p);
    return make_float2(v.x, v.y);
}
__device__ __forceinline__ double2 ldnt(const double2 *p) {
    const f64x2 v = __builtin_nontemporal_load((const f64x2 *)p);
    return make_double2(v.x, v.y);
}
__device__ __forceinline__ void stnt(float2 v, float2 *p) {
    f32x2 w;
    w.x = v.x;
    w.y = v.y;
    __builtin_nontemporal_store(w, (f32x2 *)p);
}
__device__ __forceinline__ void stnt(double2 v, double2 *p) {
    f64x2 w;
    w.x = v.x;
    w.y = v.y;
    __builtin_nontemporal_store(w, (f64x2 *)p);
}
template <typename T>
struct Vec2;
template <>
struct Vec2<double> {
    typedef double2 type;
};
template <>
struct Vec2<float> {
    typedef float2 type;
};


// FP64 -> BF16, round to nearest even, directly from the double (no double
// rounding through FP32).  Inputs are positive normal numbers well inside the
// BF16 range; the exponent carry of the rounding increment is handled by the
// integer add.
__device__ __forceinline__ bf16 f64_to_bf16_rne(double x) {
    uint64_t u = (uint64_t)__double_as_longlong(x);
    uint64_t sign = u >> 63;
    int64_t e = (int64_t)((u >> 52) & 0x7ff);
    uint64_t mant = u & 0xfffffffffffffull;
    // 8 significant bits: keep the top 7 mantissa bits, round the other 45
    uint64_t keep = mant >> 45;
    uint64_t rest = mant & ((1ull << 45) - 1);
    uint64_t half = 1ull << 44;
    if (rest > half || (rest == half && (keep & 1))) {
        keep += 1;
        if (keep == 128) {
            keep = 0;
            e += 1;
        }
    }
    int64_t eb = e - 1023 + 127;
    if (e == 0 || eb <= 0) return (bf16)(sign << 15);           // zero / underflow -> signed zero
    if (eb >= 255) return (bf16)((sign << 15) | (0xffu << 7));  // overflow -> inf
    return (bf16)((sign << 15) | ((uint64_t)eb << 7) | keep);
}

// ---------------------------------------------------------------- level views
template <typename V, typename K>
struct Lev {
    int n;           // vertices per side
    int pitch;       // elements per row
    long long plane; // n * pitch
    V s;             // h^-2
    const K *kx, *ky, *kz;
    const V *dinv;   // 1 / diagonal of A at interior vertices, 0 elsewhere
    const V *a27;    // Galerkin level: 27 coefficient arrays (d27 order), else null
    long long nel;   // elements per array (n * plane)
};

template <typename V>
struct ChebCoef {
    int m;          // steps per smoothing
    V cfirst;       // 1/theta
    V c1[MAX_DEGREE], c2[MAX_DEGREE];  // step j >= 1: rho_j rho_{j-1}, 2 rho_j / delta
};

// Per-level buffers the V-cycle uses (device-resident array of these).
template <typename V, typename K>
struct LevBuf {
    Lev<V, K> L;
    V *b, *x, *t1, *t2;
};

struct Tiling {
    int tiles_x, tiles_y, zchunk, nblocks;
};


// ---------------------------------------------------------------- value functions
// (A u)_p for one vertex from its 7 values and 6 link coefficients.
template <typename T>
__device__ __forceinline__ T apply7(T up, T uw, T ue, T us, T un, T ub, T ut, T kw, T ke, T ks, T kn,
                                    T kb, T kt, T s) {
    T acc = kw * (up - uw);
    acc = fmaT(ke, up - ue, acc);
    acc = fmaT(ks, up - us, acc);
    acc = fmaT(kn, up - un, acc);
    acc = fmaT(kb, up - ub, acc);
    acc = fmaT(kt, up - ut, acc);
    return s * acc;
}
template <typename T>
__device__ __forceinline__ T diag7(T kw, T ke, T ks, T kn, T kb, T kt, T s) {
    return s * (((kw + ke) + (ks + kn)) + (kb + kt));
}
// first Chebyshev step from x0 = 0:  x1 = (1/theta) D^-1 b, with the stored D^-1
template <typename T>
__device__ __forceinline__ T cheb_first_val(T bv, T dinv, T c) { return c * (bv * dinv); }
// Chebyshev step: x_{j+1} = x_j + c1 (x_j - x_{j-1}) + c2 D^-1 (b - A x_j)
template <typename T>
__device__ __forceinline__ T cheb_step_val(T xc, T diff, T bv, T ax, T d, T c1, T c2) {
    return fmaT(c2, (bv - ax) / d, fmaT(c1, diff, xc));
}

// Galerkin levels store 27 coefficient arrays; array d27(dx,dy,dz) holds the
// coefficient of u[p + (dx,dy,dz)] in row p.
__host__ __device__ constexpr int d27(int dx, int dy, int dz) { return (dz + 1) * 9 + (dy + 1) * 3 + (dx + 1); }
// (A u)_p of a 27-point level, summed in the fixed order dz, dy, dx.
template <typename V>
__device__ __forceinline__ V apply27_at(const V *a, long long nel, const V *u, long long o, int pitch, long long plane) {
    V acc = V(0);
#pragma unroll
    for (int dz = -1; dz <= 1; ++dz)
#pragma unroll
        for (int dy = -1; dy <= 1; ++dy)
#pragma unroll
            for (int dx = -1; dx <= 1; ++dx)
                acc = fmaT(a[(long long)d27(dx, dy, dz) * nel + o], u[o + dz * plane + dy * pitch + dx], acc);
    return acc;
}

// The 7 vertex values and 6 link coefficients around offset o, read from memory.
template <typename V, typename K>
struct Nbr {
    V up, uw, ue, us, un, ub, ut;
    V kw, ke, ks, kn, kb, kt;
};
template <typename V, typename K>
__device__ __forceinline__ void load_k(const Lev<V, K> &L, long long o, Nbr<V, K> &q) {
    q.kw = kval(L.kx[o - 1]);
    q.ke = kval(L.kx[o]);
    q.ks = kval(L.ky[o - L.pitch]);
    q.kn = kval(L.ky[o]);
    q.kb = kval(L.kz[o - L.plane]);
    q.kt = kval(L.kz[o]);
}
template <typename V, typename K>
__device__ __forceinline__ void load_u(const Lev<V, K> &L, const V *u, long long o, Nbr<V, K> &q) {
    q.up = u[o];
    q.uw = u[o - 1];
    q.ue = u[o + 1];
    q.us = u[o - L.pitch];
    q.un = u[o + L.pitch];
    q.ub = u[o - L.plane];
    q.ut = u[o + L.plane];
}
template <typename V, typename K>
__device__ __forceinline__ V apply_at(const Lev<V, K> &L, const V *u, long long o) {
    if (L.a27) return apply27_at(L.a27, L.nel, u, o, L.pitch, L.plane);
    Nbr<V, K> q;
    load_k(L, o, q);
    load_u(L, u, o, q);
    return apply7(q.up, q.uw, q.ue, q.us, q.un, q.ub, q.ut, q.kw, q.ke, q.ks, q.kn, q.kb, q.kt, L.s);
}

// ---------------------------------------------------------------- buffer addressing
// Raw buffer resources (CDNA "buffer" instructions): an array's base address
// for the current plane lives in scalar registers, each thread keeps a fixed
// 32-bit byte offset, so a load costs no vector address arithmetic.  A load
// whose offset is at or beyond the resource's byte count returns 0 and
// touches no memory (a store is dropped); kernels give vertices outside the
// grid the offset kOutside for that.
typedef __amdgpu_buffer_rsrc_t Rsrc;
constexpr int kBufDword3 = 0x00020000;      // raw buffer, 32-bit data format (descriptor word 3)
constexpr uint32_t kOutside = 0x80000000u;  // beyond every resource, also after small displacements
__device__ __forceinline__ Rsrc rsrc(const void *base, uint32_t bytes) {
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void *>(base), (short)0, (int)bytes, kBufDword3);
}
// Cache-policy bits of a streaming (nontemporal) access.  Only for data no
// other thread of the launch reads: L2 evicts such lines first, so a halo line
// that a neighbouring tile reads a little later is fetched again.  Measured on
// the one-sweep smoothers at 513^3: with the bit on their halo-bearing loads
// (links, b, D^-1, x) they fetched 1.3-1.9x their algorithmic reads; without
// it 1.1x, and ran 14-22 % faster.
constexpr int kNT = 2;
template <typename T>
struct Buf;
template <>
struct Buf<float> {
    template <int AUX = 0>
    static __device__ __forceinline__ float ld(Rsrc r, uint32_t v, uint32_t s) {
        return __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(r, v, s, AUX));
    }
    template <int AUX = 0>
    static __device__ __forceinline__ void st(float x, Rsrc r, uint32_t v, uint32_t s) {
        __builtin_amdgcn_raw_buffer_store_b32(__float_as_uint(x), r, v, s, AUX);
    }
};
template <>
struct Buf<double> {
    template <int AUX = 0>
    static __device__ __forceinline__ double ld(Rsrc r, uint32_t v, uint32_t s) {
        return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, v, s, AUX));
    }
    template <int AUX = 0>
    static __device__ __forceinline__ void st(double x, Rsrc r, uint32_t v, uint32_t s) {
        typedef decltype(__builtin_amdgcn_raw_buffer_load_b64(r, 0, 0, 0)) U64;
        __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(U64, x), r, v, s, AUX);
    }
};
template <>
struct Buf<uint16_t> {
    template <int AUX = 0>
    static __device__ __forceinline__ uint16_t ld(Rsrc r, uint32_t v, uint32_t s) {
        return __builtin_amdgcn_raw_buffer_load_b16(r, v, s, AUX);
    }
};

// ---------------------------------------------------------------- reductions
// Deterministic workgroup sum: wave64 butterfly, then the per-wave values in
// wave order.  Result valid in thread 0.
template <int NTH>
__device__ __forceinline__ double block_sum(double v) {
    __shared__ double red[NTH / 64];
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    __syncthreads();  // a previous call's reader (thread 0) is done with red[]
    if (lane == 0) red[wave] = v;
    __syncthreads();
    double s = 0.0;
    if (threadIdx.x == 0) {
#pragma unroll
        for (int w = 0; w < NTH / 64; ++w) s += red[w];
    }
    return s;
}

// ---------------------------------------------------------------- tiling
// Workgroup b runs on XCD b % 8 (dispatch is round-robin over the 8 XCDs, each
// with its own L2).  When the number of tile rows is a multiple of 8, XCD x
// owns the tile rows [x*ty/8, (x+1)*ty/8) of every z-chunk, visited x-fastest,
// then y, then z: every halo row and column except those at the slab edges is
// a line the same XCD's L2 already holds, and all XCDs stream the same band of
// planes at any moment.  Measured on MI355X at 513^3: L2 fetches within 3-8%
// of the algorithmic bytes and the speed of the plain x-fastest order (which
// fetches 30% more, cross-XCD halo lines served by the Infinity Cache);
// contiguous z-slabs per XCD were 5-11% slower (eight far-apart streams).
__device__ __forceinline__ void tile_of(int b, const Tiling &t, int &tx, int &ty, int &cz) {
    if ((t.tiles_y & 7) == 0) {
        const int rows = t.tiles_y >> 3;
        int slot = b >> 3;
        tx = slot % t.tiles_x;
        slot /= t.tiles_x;
        ty = (b & 7) * rows + slot % rows;
        cz = slot / rows;
    } else {
        tx = b % t.tiles_x;
        b /= t.tiles_x;
        ty = b % t.tiles_y;
        cz = b / t.tiles_y;
    }
}

struct Column {
    int i, j, k0, k1;
    bool active;
};
// tile -> (x tile, y tile, z chunk), x fastest; a thread owns the column
// (i, j) for planes k0..k1-1.  x tiles start at i = 0 so rows stay aligned.
__device__ __forceinline__ Column tile_column(int n, const Tiling &t) {
    int tx, ty, cz;
    tile_of(blockIdx.x, t, tx, ty, cz);
    Column c;
    c.i = tx * TX + (threadIdx.x & (TX - 1));
    c.j = 1 + ty * TY + (threadIdx.x >> 6);
    c.k0 = 1 + cz * t.zchunk;
    c.k1 = min(c.k0 + t.zchunk, n - 1);
    c.active = c.i >= 1 && c.i <= n - 2 && c.j <= n - 2 && c.k0 < c.k1;
    return c;
}

// ================================================================ stencil kernels
// Each thread marches its column in z, keeping u(k-1), u(k) and the lower
// z-link in registers; x/y neighbours come through the L1/L2 caches.

// y = A u ;  DOT: partial[wg] = sum u . (A u)   (PCG p.Ap).  u may be stored
// narrower than V (the FP32 search direction of the MIXED solve): its values
// are widened exactly before the arithmetic.
template <typename V, typename K, bool DOT, typename U = V>
__global__ __launch_bounds__(NT) void k_apply(Lev<V, K> L, Tiling t, const U *__restrict__ u,
                                              V *__restrict__ y, double *__restrict__ partial,
                                              const int *__restrict__ skip) {
    if (skip && *skip) return;
    const Column c = tile_column(L.n, t);
    double dot = 0.0;
    if (c.active) {
        const int pitch = L.pitch;
        const long long plane = L.plane;
        long long o = (long long)c.k0 * plane + (long long)c.j * pitch + c.i;
        V ub = (V)u[o - plane], up = (V)u[o];
        V kb = kval(L.kz[o - plane]);
        for (int k = c.k0; k < c.k1; ++k, o += plane) {
            const V ut = (V)u[o + plane];
            const V uw = (V)u[o - 1], ue = (V)u[o + 1], us = (V)u[o - pitch], un = (V)u[o + pitch];
            const V kw = kval(L.kx[o - 1]), ke = kval(ldnt(&L.kx[o])), ks = kval(L.ky[o - pitch]),
                    kn = kval(L.ky[o]), kt = kval(ldnt(&L.kz[o]));
            const V r = apply7(up, uw, ue, us, un, ub, ut, kw, ke, ks, kn, kb, kt, L.s);
            stnt(r, &y[o]);
            if (DOT) dot = fmaT((double)up, (double)r, dot);
            ub = up;
            up = ut;
            kb = kt;
        }
    }
    if (DOT) {
        const double s = block_sum<NT>(dot);
        if (threadIdx.x == 0) partial[blockIdx.x] = s;
    }
}

// The outer FP64 operator with two x points per lane: a tile is
// (128 WX) x (4 / WX) points of a z-chunk (WX waves side by side along x,
// each covering 128 points of a row), u and the links are read as pairs (8-
// and 16-byte loads), the west/east values at the pair's ends singly.  Per
// point the arithmetic is that of k_apply; the dot adds the pair's two terms
// in x order.  Lanes whose two points are both outside the interior load
// nothing.  WX = 4 (512 x 1 tiles) on long rows: a workgroup then reads one
// contiguous 2-4 KB segment per array and plane (measured at 513^3: 1 % faster
// than 128 x 4 tiles); WX = 1 on short rows, which would leave lanes idle.
template <bool DOT, typename U, int WX = 1>
__global__ __launch_bounds__(NT) void k_apply_x2(Lev<double, double> L, Tiling t, const U *__restrict__ u,
                                                 double *__restrict__ y, double *__restrict__ partial,
                                                 const int *__restrict__ skip) {
    static_assert(WX == 1 || WX == 2 || WX == 4, "four waves per workgroup");
    if (skip && *skip) return;
    typedef typename Vec2<U>::type U2;
    int tx, ty, cz;
    tile_of(blockIdx.x, t, tx, ty, cz);
    const int wave = (int)(threadIdx.x >> 6);
    const int i0 = (tx * WX + wave % WX) * TX2 + 2 * (int)(threadIdx.x & (TX - 1));
    const int j = 1 + ty * (TY / WX) + wave / WX;
    const int k0 = 1 + cz * t.zchunk, k1 = min(k0 + t.zchunk, L.n - 1);
    const bool a0 = i0 >= 1 && i0 <= L.n - 2, a1 = i0 + 1 <= L.n - 2;
    double dot = 0.0;
    if ((a0 || a1) && j <= L.n - 2 && k0 < k1) {
        const int pitch = L.pitch;
        const long long plane = L.plane;
        const double s = L.s;
        long long o = (long long)k0 * plane + (long long)j * pitch + i0;
        U2 ub = *(const U2 *)(u + o - plane), up = *(const U2 *)(u + o);
        double2 kb = *(const double2 *)(L.kz + o - plane);
        for (int k = k0; k < k1; ++k, o += plane) {
            const U2 ut = *(const U2 *)(u + o + plane);
            const U2 us = *(const U2 *)(u + o - pitch), un = *(const U2 *)(u + o + pitch);
            const double uw = (double)u[o - 1], ue = (double)u[o + 2];
            const double kw = L.kx[o - 1];
            const double2 ke = ldnt((const double2 *)(L.kx + o)), kt = ldnt((const double2 *)(L.kz + o));
            const double2 ks = *(const double2 *)(L.ky + o - pitch), kn = *(const double2 *)(L.ky + o);
            const double p0 = (double)up.x, p1 = (double)up.y;
            double r0 = apply7(p0, uw, p1, (double)us.x, (double)un.x, (double)ub.x, (double)ut.x, kw, ke.x, ks.x,
                               kn.x, kb.x, kt.x, s);
            double r1 = apply7(p1, p0, ue, (double)us.y, (double)un.y, (double)ub.y, (double)ut.y, ke.x, ke.y, ks.y,
                               kn.y, kb.y, kt.y, s);
            if (!a0) r0 = 0.0;
            if (!a1) r1 = 0.0;
            stnt(make_double2(r0, r1), (double2 *)(y + o));
            if (DOT) {
                dot = fmaT(p0, r0, dot);
                dot = fmaT(p1, r1, dot);
            }
            ub = up;
            up = ut;
            kb = kt;
        }
    }
    if (DOT) {
        const double sum = block_sum<NT>(dot);
        if (threadIdx.x == 0) partial[blockIdx.x] = sum;
    }
}

// r = b - A u   (FP64 true residual and the x0 != 0 start)
template <typename V, typename K>
__global__ __launch_bounds__(NT) void k_residual(Lev<V, K> L, Tiling t, const V *__restrict__ b,
                                                 const V *__restrict__ u, V *__restrict__ r,
                                                 const int *__restrict__ skip) {
    if (skip && *skip) return;
    const Column c = tile_column(L.n, t);
    if (!c.active) return;
    const int pitch = L.pitch;
    const long long plane = L.plane;
    long long o = (long long)c.k0 * plane + (long long)c.j * pitch + c.i;
    V ub = u[o - plane], up = u[o];
    V kb = kval(L.kz[o - plane]);
    for (int k = c.k0; k < c.k1; ++k, o += plane) {
        const V ut = u[o + plane];
        const V uw = u[o - 1], ue = u[o + 1], us = u[o - pitch], un = u[o + pitch];
        const V kw = kval(L.kx[o - 1]), ke = kval(ldnt(&L.kx[o])), ks = kval(L.ky[o - pitch]),
                kn = kval(L.ky[o]), kt = kval(ldnt(&L.kz[o]));
        stnt(ldnt(&b[o]) - apply7(up, uw, ue, us, un, ub, ut, kw, ke, ks, kn, kb, kt, L.s), &r[o]);
        ub = up;
        up = ut;
        kb = kt;
    }
}

// First Chebyshev step from zero: x1 = c D^-1 b.
// CVT (finest level, mixed precision): b is converted from the FP64 residual
// r64 and also stored (b_out) for the later sweeps of the cycle.
template <typename V, typename K, bool CVT>
__global__ __launch_bounds__(NT) void k_cheb_first(Lev<V, K> L, Tiling t, const V *__restrict__ b,
                                                   const double *__restrict__ r64, V *__restrict__ b_out,
                                                   V *__restrict__ x_out, V c, const int *__restrict__ skip) {
    if (skip && *skip) return;
    const Column col = tile_column(L.n, t);
    if (!col.active) return;
    long long o = (long long)col.k0 * L.plane + (long long)col.j * L.pitch + col.i;
    for (int k = col.k0; k < col.k1; ++k, o += L.plane) {
        V bv;
        if (CVT) {
            bv = (V)ldnt(&r64[o]);
            stnt(bv, &b_out[o]);
        } else {
            bv = ldnt(&b[o]);
        }
        stnt(cheb_first_val(bv, ldnt(&L.dinv[o]), c), &x_out[o]);
    }
}

// The first two Chebyshev steps from zero in one sweep: x1 = c0 D^-1 b is
// evaluated on the fly at the stencil points (it is pointwise), and
//   x2 = x1 + c1 x1 + c2 D^-1 (b - A x1).
// Same values as k_cheb_first followed by the PM = 1 step.  WX1 also stores
// x1 (needed as the previous iterate when the degree exceeds 2).  Each thread
// owns two adjacent rows j, j+1 of a 64 x 8 tile (tiling with TY_PRE rows), so
// x1 is evaluated on rows j-1 .. j+2 for two outputs instead of three rows
// per output; 7 % faster at 513^3 than one row per thread.
template <typename V, typename K, bool WX1>
__global__ __launch_bounds__(NT) void k_cheb_pre2(Lev<V, K> L, Tiling t, const V *__restrict__ b,
                                                  V *__restrict__ out, V *__restrict__ x1out, V c0, V c1, V c2,
                                                  const int *__restrict__ skip) {
    if (skip && *skip) return;
    int tx, ty, cz;
    tile_of(blockIdx.x, t, tx, ty, cz);
    const int i = tx * TX + (int)(threadIdx.x & (TX - 1));
    const int j = 1 + ty * TY_PRE + 2 * (int)(threadIdx.x >> 6);
    const int k0 = 1 + cz * t.zchunk, k1 = min(k0 + t.zchunk, L.n - 1);
    if (i < 1 || i > L.n - 2 || j > L.n - 2 || k0 >= k1) return;
    const bool row1 = j + 1 <= L.n - 2;  // second row interior (rows up to j+2 are in the array)
    const int pitch = L.pitch;
    const long long plane = L.plane;
    const V *__restrict__ dv = L.dinv;
    long long o = (long long)k0 * plane + (long long)j * pitch + i;
    const long long q = pitch;  // offset of row j+1
    V ub0 = cheb_first_val(b[o - plane], dv[o - plane], c0), ub1 = cheb_first_val(b[o + q - plane], dv[o + q - plane], c0);
    V bp0 = b[o], bp1 = b[o + q];
    V up0 = cheb_first_val(bp0, dv[o], c0), up1 = cheb_first_val(bp1, dv[o + q], c0);
    V kb0 = kval(L.kz[o - plane]), kb1 = kval(L.kz[o + q - plane]);
    for (int k = k0; k < k1; ++k, o += plane) {
        const V bt0 = b[o + plane], bt1 = b[o + q + plane];
        const V ut0 = cheb_first_val(bt0, dv[o + plane], c0), ut1 = cheb_first_val(bt1, dv[o + q + plane], c0);
        const V us0 = cheb_first_val(b[o - pitch], dv[o - pitch], c0);
        const V un1 = cheb_first_val(b[o + q + pitch], dv[o + q + pitch], c0);
        const V uw0 = cheb_first_val(b[o - 1], dv[o - 1], c0), ue0 = cheb_first_val(b[o + 1], dv[o + 1], c0);
        const V uw1 = cheb_first_val(b[o + q - 1], dv[o + q - 1], c0),
                ue1 = cheb_first_val(b[o + q + 1], dv[o + q + 1], c0);
        const V kw0 = kval(L.kx[o - 1]), ke0 = kval(ldnt(&L.kx[o])), kw1 = kval(L.kx[o + q - 1]),
                ke1 = kval(ldnt(&L.kx[o + q]));
        const V ks0 = kval(L.ky[o - pitch]), kmid = kval(L.ky[o]), kn1 = kval(L.ky[o + q]);
        const V kt0 = kval(ldnt(&L.kz[o])), kt1 = kval(ldnt(&L.kz[o + q]));
        {
            const V ax = apply7(up0, uw0, ue0, us0, up1, ub0, ut0, kw0, ke0, ks0, kmid, kb0, kt0, L.s);
            const V d = diag7(kw0, ke0, ks0, kmid, kb0, kt0, L.s);
            stnt(cheb_step_val(up0, up0, bp0, ax, d, c1, c2), &out[o]);
            if (WX1) stnt(up0, &x1out[o]);
        }
        if (row1) {
            const V ax = apply7(up1, uw1, ue1, up0, un1, ub1, ut1, kw1, ke1, kmid, kn1, kb1, kt1, L.s);
            const V d = diag7(kw1, ke1, kmid, kn1, kb1, kt1, L.s);
            stnt(cheb_step_val(up1, up1, bp1, ax, d, c1, c2), &out[o + q]);
            if (WX1) stnt(up1, &x1out[o + q]);
        }
        ub0 = up0;
        up0 = ut0;
        ub1 = up1;
        up1 = ut1;
        bp0 = bt0;
        bp1 = bt1;
        kb0 = kt0;
        kb1 = kt1;
    }
}

// D^-1 at the interior vertices of a level (setup).
template <typename V, typename K>
__global__ __launch_bounds__(NT) void k_dinv(Lev<V, K> L, Tiling t, V *__restrict__ dinv) {
    const Column col = tile_column(L.n, t);
    if (!col.active) return;
    long long o = (long long)col.k0 * L.plane + (long long)col.j * L.pitch + col.i;
    for (int k = col.k0; k < col.k1; ++k, o += L.plane) {
        const V d = diag7(kval(L.kx[o - 1]), kval(L.kx[o]), kval(L.ky[o - L.pitch]), kval(L.ky[o]),
                          kval(L.kz[o - L.plane]), kval(L.kz[o]), L.s);
        dinv[o] = V(1) / d;
    }
}

// Chebyshev step  out = x + c1 (x - x_prev) + c2 D^-1 (b - A x).
// PM = 0: no previous iterate (c1 term vanishes); PM = 1: previous iterate is
// zero (diff = x); PM = 2: previous iterate in xp.  out may alias xp (read only
// at the thread's own vertex before the write), never x.
// DOTR: last sweep of the cycle on the finest level; partial[wg] = sum r64 . out.
template <typename V, typename K, int PM, bool DOTR>
__global__ __launch_bounds__(NT) void k_cheb_step(Lev<V, K> L, Tiling t, const V *__restrict__ b,
                                                  const V *__restrict__ x, const V *xp, V *out, V c1, V c2,
                                                  const double *__restrict__ r64, double *__restrict__ partial,
                                                  const int *__restrict__ skip,
                                                  const double *__restrict__ q64 = nullptr) {
    if (skip && *skip) return;
    const Column col = tile_column(L.n, t);
    double dot = 0.0, dotq = 0.0;
    if (col.active) {
        const int pitch = L.pitch;
        const long long plane = L.plane;
        long long o = (long long)col.k0 * plane + (long long)col.j * pitch + col.i;
        V ub = x[o - plane], up = x[o];
        V kb = kval(L.kz[o - plane]);
        for (int k = col.k0; k < col.k1; ++k, o += plane) {
            const V ut = x[o + plane];
            const V uw = x[o - 1], ue = x[o + 1], us = x[o - pitch], un = x[o + pitch];
            const V kw = kval(L.kx[o - 1]), ke = kval(ldnt(&L.kx[o])), ks = kval(L.ky[o - pitch]),
                    kn = kval(L.ky[o]), kt = kval(ldnt(&L.kz[o]));
            const V ax = apply7(up, uw, ue, us, un, ub, ut, kw, ke, ks, kn, kb, kt, L.s);
            const V d = diag7(kw, ke, ks, kn, kb, kt, L.s);
            const V diff = PM == 0 ? V(0) : PM == 1 ? up : up - ldnt(&xp[o]);
            const V v = cheb_step_val(up, diff, ldnt(&b[o]), ax, d, PM == 0 ? V(0) : c1, c2);
            stnt(v, &out[o]);
            if (DOTR) {
                dot = fmaT(ldnt(&r64[o]), (double)v, dot);
                if (q64) dotq = fmaT(ldnt(&q64[o]), (double)v, dotq);
            }
            ub = up;
            up = ut;
            kb = kt;
        }
    }
    if (DOTR) {
        const double s = block_sum<NT>(dot);
        if (threadIdx.x == 0) partial[blockIdx.x] = s;
        if (q64) {  // flexible CG: second partial array q.z after the first
            const double sq = block_sum<NT>(dotq);
            if (threadIdx.x == 0) partial[gridDim.x + blockIdx.x] = sq;
        }
    }
}

// Post-smoothing by a degree-2 Chebyshev polynomial in one sweep (7-point
// link levels):
//   x1 = x0 + c0 D^-1 (b - A x0),   x2 = x1 + c1 (x1 - x0) + c2 D^-1 (b - A x1),
// with the arithmetic of a k_cheb_step with PM = 0 followed by one with PM = 2,
// so x2 is the same to the bit.  x1 never goes to memory.  A workgroup owns a
// 64 x ROWS tile (one vertex per thread, one tile row per wave) and marches up
// its z-chunk in phases m = k0-1 .. k1, one barrier each.  In phase m it
//   * computes x1 of plane m at its own vertex from x0 of planes m-1 .. m+1,
//   * on the last waves, computes x1 of plane m on a one-point ring around
//     the tile (recomputed by the neighbouring tiles too),
//   * computes x2 of plane m-1 from x1 of planes m-2 .. m,
//   * stages x0 of plane m+2 (tile and a two-point ring).
// x0 and x1 are kept in four-plane LDS ring buffers, so a thread holds no
// plane history in registers: what it holds are the loads in flight for the
// next phase (the links and b of plane m+1, x0 of plane m+3), which keeps the
// register count, and with it the number of resident workgroups, up.  The
// phase body is unrolled four times, so every LDS slot and register set is
// named at compile time (slot = plane - k0 + 1 mod 4).  Loads go through one
// buffer resource per array and chunk, the plane chosen by the scalar offset,
// each thread with a fixed byte offset: no vector address arithmetic; a
// vertex outside the grid gets an offset beyond every resource and reads 0.
// The loads the ring and halo share with neighbouring tiles use the plain
// cache policy, so those tiles find the lines in L2; only r64 and q64 are
// streamed nontemporal.  The diagonal of a vertex is formed once and serves
// both steps.  One read of
// x0, b and the links and one write of x2 replace the two sweeps' reads of x0
// (twice), b and the links (twice) and the write and read of x1.  out must not
// alias x0 (other tiles read x0 in their rings).  DOTR 1: partial[wg] =
// sum r64 . x2; DOTR 2: and sum q64 . x2 after it.
template <typename V, typename K, int DOTR, int ROWS>
__global__ __launch_bounds__(TX * ROWS) void k_post2(Lev<V, K> L, Tiling t, const V *__restrict__ b,
                                                   const V *__restrict__ x0, V *__restrict__ out, V c0, V c1, V c2,
                                                   const double *__restrict__ r64, double *__restrict__ partial,
                                                   const int *__restrict__ skip,
                                                   const double *__restrict__ q64 = nullptr) {
    constexpr int W = TX, H = ROWS, NTH = TX * ROWS;
    constexpr int XW = W + 4, YW = W + 2;       // row lengths of the x0 and x1 tiles
    constexpr int HALO0 = 4 * XW + 4 * H;       // two-point ring of the x0 tile
    constexpr int RING = 2 * YW + 2 * H;        // one-point ring of the x1 tile
    constexpr int RING0 = NTH - RING;           // first thread of the ring
    static_assert(HALO0 <= NTH && RING <= NTH, "one pass per ring");
    constexpr uint32_t SV = sizeof(V), SK = sizeof(K);
    __shared__ V sx0[4][H + 4][XW];  // x0 by plane slot, tile at [2, H+1] x [2, W+1]
    __shared__ V sx1[4][H + 2][YW];  // x1 by plane slot, tile at [1, H] x [1, W]
    if (skip && *skip) return;
    int tx, ty, cz;
    tile_of(blockIdx.x, t, tx, ty, cz);
    const int lx = (int)(threadIdx.x & (W - 1)), ly = (int)(threadIdx.x >> 6);
    const int wave = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    const int i0 = tx * W, j0 = 1 + ty * H;  // grid position of tile point (0, 0)
    const int i = i0 + lx, j = j0 + ly;
    const int n = L.n, pitch = L.pitch;
    const long long plane = L.plane;
    const int k0 = 1 + cz * t.zchunk, k1 = min(k0 + t.zchunk, n - 1);
    if (k0 >= k1) return;  // uniform over the workgroup
    const int np = k1 - k0 + 2;  // phases
    auto in_xy = [n](int a, int c) { return (unsigned)a < (unsigned)n && (unsigned)c < (unsigned)n; };
    auto inner_xy = [n](int a, int c) { return a >= 1 && a <= n - 2 && c >= 1 && c <= n - 2; };
    const bool own_inner = inner_xy(i, j);
    const uint32_t own = (uint32_t)(j * pitch + i);
    const uint32_t ox0 = in_xy(i, j) ? own * SV : kOutside;     // x0 of the own vertex
    const uint32_t ok = own_inner ? own * SK : kOutside;         // its links
    const uint32_t ov = own_inner ? own * SV : kOutside;         // its b and x2
    const uint32_t o8 = own_inner ? own * 8u : kOutside;         // its r64, q64
    // x0 ring slot of this thread (threads 0 .. HALO0-1): two rows above and
    // below the tile, two columns left and right of it
    const int h = (int)threadIdx.x;
    int hy = 0, hx = 0;
    if (h < 4 * XW) {
        const int r = h / XW;
        hy = r < 2 ? r : r + H;
        hx = h % XW;
    } else {
        const int r = h - 4 * XW;
        hy = 2 + r / 4;
        hx = (r & 3) < 2 ? (r & 3) : (r & 3) + W;
    }
    const bool hal = h < HALO0;
    const uint32_t ohal =
        (hal && in_xy(i0 - 2 + hx, j0 - 2 + hy)) ? (uint32_t)((j0 - 2 + hy) * pitch + (i0 - 2 + hx)) * SV : kOutside;
    // x1 ring slot (threads RING0 .. NTH-1): one row above and below, one
    // column left and right
    const int g = h - RING0;
    int gy = 1, gx = 1;  // a valid slot for threads outside the ring
    if (g < 0) {
    } else if (g < 2 * YW) {
        gy = g < YW ? 0 : H + 1;
        gx = g % YW;
    } else {
        const int q = g - 2 * YW;
        gy = 1 + q / 2;
        gx = (q & 1) ? W + 1 : 0;
    }
    const bool rng = g >= 0;
    const bool rng_inner = rng && inner_xy(i0 - 1 + gx, j0 - 1 + gy);
    const uint32_t rpt = (uint32_t)((j0 - 1 + gy) * pitch + (i0 - 1 + gx));
    const uint32_t rk = rng_inner ? rpt * SK : kOutside, rv = rng_inner ? rpt * SV : kOutside;
    const bool ring_wave = wave >= RING0 / 64;  // uniform: this wave holds ring threads

    // One resource per array for the whole chunk, based at plane mb = k0-2
    // (kx one element back: kx[o-1] at offset o; ky one row back: ky[o-pitch]
    // at o); plane m is reached through the scalar offset (m - mb) * plane
    // bytes.  The byte count admits every offset below kOutside.
    const long long mb = (long long)(k0 - 2) * plane;
    constexpr uint32_t kAll = 0x7fffffffu;
    const Rsrc rx0 = rsrc(x0 + mb, kAll), rb = rsrc(b + mb, kAll), rout = rsrc(out + mb, kAll);
    const Rsrc rkx = rsrc(L.kx + (mb - 1), kAll), rky = rsrc(L.ky + (mb - pitch), kAll), rkz = rsrc(L.kz + mb, kAll);
    const Rsrc rr64 = rsrc(r64 + mb, kAll), rq64 = rsrc(q64 ? q64 + mb : r64 + mb, kAll);
    const uint32_t pbv = (uint32_t)plane * SV, pbk = (uint32_t)plane * SK, pb8 = (uint32_t)plane * 8u;
    auto uni = [](uint32_t v) { return (uint32_t)__builtin_amdgcn_readfirstlane((int)v); };  // keep in a scalar
    // x0 of plane m (0 outside the grid); planes are passed as m - mb
    auto x0_at = [&](int m, uint32_t off) -> V {
        return (m >= 0 && m < n) ? Buf<V>::ld(rx0, off, uni((uint32_t)(m - k0 + 2)) * pbv) : V(0);
    };
    struct Raw {  // a vertex's links (without the one below) and b at one plane, as stored
        K kw, ke, ks, kn, kt;
        V bv;
    };
    auto load_raw = [&](int m, uint32_t okk, uint32_t ovv, Raw &r) {
        const uint32_t pl = uni((uint32_t)(m - k0 + 2)), sk = pl * pbk, sv = pl * pbv;
        r.kw = Buf<K>::ld(rkx, okk, sk);
        r.ke = Buf<K>::ld(rkx, okk + SK, sk);
        r.ks = Buf<K>::ld(rky, okk, sk);
        r.kn = Buf<K>::ld(rky, okk + (uint32_t)pitch * SK, sk);
        r.kt = Buf<K>::ld(rkz, okk, sk);
        r.bv = Buf<V>::ld(rb, ovv, sv);
    };
    struct Lk {  // the same widened, with the link below and the diagonal
        V kw, ke, ks, kn, kb, kt, bv, d;
    };
    auto widen = [&](const Raw &r, V kb, Lk &w) {
        w.kw = kval(r.kw);
        w.ke = kval(r.ke);
        w.ks = kval(r.ks);
        w.kn = kval(r.kn);
        w.kb = kb;
        w.kt = kval(r.kt);
        w.bv = r.bv;
        w.d = diag7(w.kw, w.ke, w.ks, w.kn, w.kb, w.kt, L.s);
    };

    // plane-indexed state: x0 and x1 of plane m live in LDS slot
    // (m - k0 + 1) & 3, the links and b of plane m in register set & 1
    Lk lk[2];   // own links, b and diagonal
    double R64[2] = {0.0, 0.0}, Q64[2] = {0.0, 0.0};
    V rkt[2];   // ring vertex: its upper z-link, widened
    Raw ro, rr;  // own / ring raw links and b of the next plane
    V xp, hp;   // the thread's x0 (own, ring slot) of the next plane to stage
    double dot = 0.0, dotq = 0.0;

    // prologue: x0 of planes k0-2 .. k0 into LDS (the ring from k0-1), x0 of
    // plane k0+1 into registers, the links of plane k0-1 (own) and k0 (ring)
    {
        const V a0 = x0_at(k0 - 2, ox0), a1 = x0_at(k0 - 1, ox0), a2 = x0_at(k0, ox0);
        const V h1 = x0_at(k0 - 1, ohal), h2 = x0_at(k0, ohal);
        sx0[3][ly + 2][lx + 2] = a0;
        sx0[0][ly + 2][lx + 2] = a1;
        sx0[1][ly + 2][lx + 2] = a2;
        if (hal) {
            sx0[0][hy][hx] = h1;
            sx0[1][hy][hx] = h2;
        }
    }
    xp = x0_at(k0 + 1, ox0);
    hp = x0_at(k0 + 1, ohal);
    load_raw(k0 - 1, ok, ov, ro);
    lk[1].kt = (k0 - 2 >= 0) ? kval(Buf<K>::ld(rkz, ok, 0)) : V(0);
    rkt[0] = kval(Buf<K>::ld(rkz, rk, pbk));
    load_raw(k0, rk, rv, rr);
    __syncthreads();

    // phase p = m - k0 + 1 with slot index Q = p & 3; returns true after the last phase
    auto phase = [&](auto QQ, int p) __attribute__((always_inline)) -> bool {
        constexpr int Q = decltype(QQ)::value;
        constexpr int P = Q & 1, QB = (Q + 3) & 3, QT = (Q + 1) & 3, QBB = (Q + 2) & 3;
        const int m = k0 - 1 + p;
        // x1 of plane m at the own vertex (0 on boundary planes and vertices)
        Lk &cw = lk[P];
        widen(ro, lk[P ^ 1].kt, cw);
        V x1m;
        {
            const V(*t0)[XW] = sx0[Q];
            const V xc = t0[ly + 2][lx + 2];
            const V ax = apply7(xc, t0[ly + 2][lx + 1], t0[ly + 2][lx + 3], t0[ly + 1][lx + 2], t0[ly + 3][lx + 2],
                                sx0[QB][ly + 2][lx + 2], sx0[QT][ly + 2][lx + 2], cw.kw, cw.ke, cw.ks, cw.kn, cw.kb,
                                cw.kt, L.s);
            const V v = cheb_step_val(xc, V(0), cw.bv, ax, cw.d, V(0), c0);
            x1m = (own_inner && m >= 1 && m <= n - 2) ? v : V(0);
        }
        if (p + 1 < np) load_raw(m + 1, ok, ov, ro);
        // r64 (q64) of plane m for the dot of x2(m) in the next phase
        if (DOTR && p >= 1 && p + 1 < np) {
            R64[P] = Buf<double>::template ld<kNT>(rr64, o8, uni((uint32_t)(p + 1)) * pb8);
            if (DOTR == 2) Q64[P] = Buf<double>::template ld<kNT>(rq64, o8, uni((uint32_t)(p + 1)) * pb8);
        }
        // planes k0-1 .. k1-1: own x1 into LDS (the history of x2 and, from
        // k0 on, the in-plane neighbours with the ring)
        if (p + 1 < np) sx1[Q][ly + 1][lx + 1] = x1m;
        if (p >= 1 && p + 1 < np && ring_wave) {
            Lk w;
            widen(rr, rkt[P ^ 1], w);
            rkt[P] = w.kt;
            const V(*t0)[XW] = sx0[Q];
            const int ry = gy + 1, rx = gx + 1;
            const V xc = t0[ry][rx];
            const V ax = apply7(xc, t0[ry][rx - 1], t0[ry][rx + 1], t0[ry - 1][rx], t0[ry + 1][rx], sx0[QB][ry][rx],
                                sx0[QT][ry][rx], w.kw, w.ke, w.ks, w.kn, w.kb, w.kt, L.s);
            const V v = cheb_step_val(xc, V(0), w.bv, ax, w.d, V(0), c0);
            if (rng) sx1[Q][gy][gx] = rng_inner ? v : V(0);
            if (p + 2 < np) load_raw(m + 1, rk, rv, rr);
        }
        // x2 of plane m-1
        if (p >= 2) {
            const Lk &pw = lk[P ^ 1];
            const V(*t1)[YW] = sx1[QB];
            const V x1c = t1[ly + 1][lx + 1];
            const V ax = apply7(x1c, t1[ly + 1][lx], t1[ly + 1][lx + 2], t1[ly][lx + 1], t1[ly + 2][lx + 1],
                                sx1[QBB][ly + 1][lx + 1], x1m, pw.kw, pw.ke, pw.ks, pw.kn, pw.kb, pw.kt, L.s);
            const V diff = x1c - sx0[QB][ly + 2][lx + 2];
            const V v = own_inner ? cheb_step_val(x1c, diff, pw.bv, ax, pw.d, c1, c2) : V(0);
            Buf<V>::template st<kNT>(v, rout, ov, uni((uint32_t)p) * pbv);
            if (DOTR) {
                dot = fmaT(R64[P ^ 1], (double)v, dot);
                if (DOTR == 2) dotq = fmaT(Q64[P ^ 1], (double)v, dotq);
            }
        }
        // x0 of plane m+2 into LDS (its ring only up to plane k1), x0 of
        // plane m+3 into registers
        if (p + 3 <= np + 1) sx0[QBB][ly + 2][lx + 2] = xp;
        if (p + 3 <= np && hal) sx0[QBB][hy][hx] = hp;
        if (p + 4 <= np + 1) xp = x0_at(m + 3, ox0);
        if (p + 4 <= np) hp = x0_at(m + 3, ohal);
        __syncthreads();
        return p + 1 == np;
    };
    for (int p = 0;; p += 4) {
        if (phase(std::integral_constant<int, 0>{}, p)) break;
        if (phase(std::integral_constant<int, 1>{}, p + 1)) break;
        if (phase(std::integral_constant<int, 2>{}, p + 2)) break;
        if (phase(std::integral_constant<int, 3>{}, p + 3)) break;
    }
    if (DOTR) {
        const double sm = block_sum<NTH>(dot);
        if (threadIdx.x == 0) partial[blockIdx.x] = sm;
        if (DOTR == 2) {
            const double sq = block_sum<NTH>(dotq);
            if (threadIdx.x == 0) partial[gridDim.x + blockIdx.x] = sq;
        }
    }
}

// Pre-smoothing by a degree-2 Chebyshev polynomial from x0 = 0 and the
// residual that follows it, in one sweep (7-point link levels):
//   x1 = c0 D^-1 b,   x2 = x1 + c1 x1 + c2 D^-1 (b - A x1),   r = b - A x2,
// with the arithmetic of k_cheb_pre2 (x1 from the stored D^-1, x2's diagonal
// from the links) and of k_residual_zr (r reduced along z on the fly: for each
// coarse plane K of the chunk, s(i,j,K) = r(2K-1)/4 + r(2K)/2 + r(2K+1)/4), so
// x2 and s are the same to the bit.  x1 never goes to memory and x2 is only
// written, never read back.  A workgroup owns a 64 x ROWS tile (one vertex per
// thread, one tile row per wave) and marches its z-chunk (even length, first
// plane odd, one residual plane beyond its end as in k_residual_zr) in phases
// m = k0-1 .. kend+1, one barrier each.  In phase m it
//   * computes x2 of plane m at its own vertex, and on the last waves on a
//     one-point ring around the tile (recomputed by the neighbouring tiles),
//     from x1 of planes m-1 .. m+1,
//   * computes r of plane m-1 at its own vertex from x2 of planes m-2 .. m
//     and adds it to the z-sum,
//   * stages x1 of plane m+2 (tile and a two-point ring; pointwise from b and
//     D^-1).
// x1 and x2 live in four-plane LDS ring buffers (slot = plane - k0 + 1 mod 4),
// the own vertex's b in a four-plane register ring; the links of the next
// plane (and the ring vertex's b) and b, D^-1 of the plane staged next are
// loaded a phase before their use.  The phase
// body is unrolled four times so that every slot is named at compile time;
// loads go through one buffer resource per array and chunk, with the plain
// cache policy (neighbouring tiles re-read the ring and halo lines from L2).
// x2 planes k0-1,
// k1 and k1+1 belong to the neighbouring chunks and are recomputed, not
// stored.  One read of b, D^-1 and the links and one write of x2 and the
// z-sums replace the two sweeps' reads of b (twice), D^-1, the links (twice)
// and x2 and the write of x2.
template <typename V, typename K, int ROWS>
__global__ __launch_bounds__(TX * ROWS) void k_pre2_res(Lev<V, K> L, Tiling t, const V *__restrict__ b,
                                                      V *__restrict__ out, V *__restrict__ zs, V c0, V c1, V c2,
                                                      const int *__restrict__ skip) {
    constexpr int W = TX, H = ROWS, NTH = TX * ROWS;
    constexpr int XW = W + 4, YW = W + 2;       // row lengths of the x1 and x2 tiles
    constexpr int HALO1 = 4 * XW + 4 * H;       // two-point ring of the x1 tile
    constexpr int RING = 2 * YW + 2 * H;        // one-point ring of the x2 tile
    constexpr int RING0 = NTH - RING;           // first thread of the ring
    static_assert(HALO1 <= NTH && RING <= NTH, "one pass per ring");
    constexpr uint32_t SV = sizeof(V), SK = sizeof(K);
    __shared__ V sx1[4][H + 4][XW];  // x1 by plane slot, tile at [2, H+1] x [2, W+1]
    __shared__ V sx2[4][H + 2][YW];  // x2 by plane slot, tile at [1, H] x [1, W]
    if (skip && *skip) return;
    int tx, ty, cz;
    tile_of(blockIdx.x, t, tx, ty, cz);
    const int lx = (int)(threadIdx.x & (W - 1)), ly = (int)(threadIdx.x >> 6);
    const int wave = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    const int i0 = tx * W, j0 = 1 + ty * H;  // grid position of tile point (0, 0)
    const int i = i0 + lx, j = j0 + ly;
    const int n = L.n, pitch = L.pitch;
    const long long plane = L.plane;
    const int k0 = 1 + cz * t.zchunk, k1 = min(k0 + t.zchunk, n - 1);
    if (k0 >= k1) return;  // uniform over the workgroup
    const int kend = min(k1, n - 2);  // last residual plane (odd)
    const int np = kend - k0 + 3;     // phases: m = k0-1 .. kend+1
    auto in_xy = [n](int a, int c) { return (unsigned)a < (unsigned)n && (unsigned)c < (unsigned)n; };
    auto inner_xy = [n](int a, int c) { return a >= 1 && a <= n - 2 && c >= 1 && c <= n - 2; };
    const bool own_inner = inner_xy(i, j);
    const uint32_t own = (uint32_t)(j * pitch + i);
    const uint32_t ovx = in_xy(i, j) ? own * SV : kOutside;  // own b, D^-1 for x1 (0 outside the grid)
    const uint32_t ok = own_inner ? own * SK : kOutside;     // own links
    const uint32_t ov = own_inner ? own * SV : kOutside;     // own x2, z-sums
    // x1 ring slot of this thread (threads 0 .. HALO1-1)
    const int h = (int)threadIdx.x;
    int hy = 0, hx = 0;
    if (h < 4 * XW) {
        const int r = h / XW;
        hy = r < 2 ? r : r + H;
        hx = h % XW;
    } else {
        const int r = h - 4 * XW;
        hy = 2 + r / 4;
        hx = (r & 3) < 2 ? (r & 3) : (r & 3) + W;
    }
    const bool hal = h < HALO1;
    const uint32_t ohal =
        (hal && in_xy(i0 - 2 + hx, j0 - 2 + hy)) ? (uint32_t)((j0 - 2 + hy) * pitch + (i0 - 2 + hx)) * SV : kOutside;
    // x2 ring slot (threads RING0 .. NTH-1)
    const int g = h - RING0;
    int gy = 1, gx = 1;  // a valid slot for threads outside the ring
    if (g < 0) {
    } else if (g < 2 * YW) {
        gy = g < YW ? 0 : H + 1;
        gx = g % YW;
    } else {
        const int q = g - 2 * YW;
        gy = 1 + q / 2;
        gx = (q & 1) ? W + 1 : 0;
    }
    const bool rng = g >= 0;
    const bool rng_inner = rng && inner_xy(i0 - 1 + gx, j0 - 1 + gy);
    const uint32_t rpt = (uint32_t)((j0 - 1 + gy) * pitch + (i0 - 1 + gx));
    const uint32_t rk = rng_inner ? rpt * SK : kOutside, rv = rng_inner ? rpt * SV : kOutside;
    const bool ring_wave = wave >= RING0 / 64;  // uniform: this wave holds ring threads

    // One resource per array for the chunk, based at plane k0-2; plane m at
    // the scalar offset (m - k0 + 2) * plane bytes
    const long long mb = (long long)(k0 - 2) * plane;
    constexpr uint32_t kAll = 0x7fffffffu;
    const Rsrc rb = rsrc(b + mb, kAll), rdv = rsrc(L.dinv + mb, kAll), rout = rsrc(out + mb, kAll);
    const Rsrc rkx = rsrc(L.kx + (mb - 1), kAll), rky = rsrc(L.ky + (mb - pitch), kAll), rkz = rsrc(L.kz + mb, kAll);
    const uint32_t pbv = (uint32_t)plane * SV, pbk = (uint32_t)plane * SK;
    auto uni = [](uint32_t v) { return (uint32_t)__builtin_amdgcn_readfirstlane((int)v); };
    auto pl = [&](int m) { return uni((uint32_t)(m - k0 + 2)); };
    // x1 of plane m at in-plane offset off (0 outside the grid or on planes past it)
    struct BD {
        V bv, dv;
    };
    auto load_bd = [&](int m, uint32_t off) -> BD {
        BD r{V(0), V(0)};
        if (m >= 0 && m < n) {
            r.bv = Buf<V>::ld(rb, off, pl(m) * pbv);
            r.dv = Buf<V>::ld(rdv, off, pl(m) * pbv);
        }
        return r;
    };
    struct Raw {  // a vertex's links (without the one below) at one plane, as stored
        K kw, ke, ks, kn, kt;
    };
    auto load_raw = [&](int m, uint32_t okk, Raw &r) {
        const uint32_t sk = pl(m) * pbk;
        r.kw = Buf<K>::ld(rkx, okk, sk);
        r.ke = Buf<K>::ld(rkx, okk + SK, sk);
        r.ks = Buf<K>::ld(rky, okk, sk);
        r.kn = Buf<K>::ld(rky, okk + (uint32_t)pitch * SK, sk);
        r.kt = Buf<K>::ld(rkz, okk, sk);
    };
    struct Lk {  // widened, with the link below and the diagonal
        V kw, ke, ks, kn, kb, kt, d;
    };
    auto widen = [&](const Raw &r, V kb, Lk &w) {
        w.kw = kval(r.kw);
        w.ke = kval(r.ke);
        w.ks = kval(r.ks);
        w.kn = kval(r.kn);
        w.kb = kb;
        w.kt = kval(r.kt);
        w.d = diag7(w.kw, w.ke, w.ks, w.kn, w.kb, w.kt, L.s);
    };

    // plane-indexed state: x1, x2 of plane m in LDS slot (m - k0 + 1) & 3, the
    // own b of plane m in bq[(m - k0 + 1) & 3], links in lk[(m - k0 + 1) & 1]
    V bq[4];
    Lk lk[2];
    V rkt[2];          // ring vertex: its upper z-link, widened
    Raw ro, rr;        // own / ring raw links of the next plane
    V rbv = V(0);      // ring vertex: b of the next plane
    BD xp, hp;         // b, D^-1 of the plane to stage next (own, x1 ring slot)
    V acc = V(0);      // z-sum of the open coarse plane

    // prologue: x1 of planes k0-2 .. k0 (own; ring from k0-1), b, D^-1 of
    // plane k0+1, the links of plane k0-1 (own) and k0 (ring)
    {
        const BD a0 = load_bd(k0 - 2, ovx), a1 = load_bd(k0 - 1, ovx), a2 = load_bd(k0, ovx);
        const BD h1 = load_bd(k0 - 1, ohal), h2 = load_bd(k0, ohal);
        sx1[3][ly + 2][lx + 2] = cheb_first_val(a0.bv, a0.dv, c0);
        sx1[0][ly + 2][lx + 2] = cheb_first_val(a1.bv, a1.dv, c0);
        sx1[1][ly + 2][lx + 2] = cheb_first_val(a2.bv, a2.dv, c0);
        if (hal) {
            sx1[0][hy][hx] = cheb_first_val(h1.bv, h1.dv, c0);
            sx1[1][hy][hx] = cheb_first_val(h2.bv, h2.dv, c0);
        }
        bq[0] = a1.bv;
        bq[1] = a2.bv;
    }
    xp = load_bd(k0 + 1, ovx);
    hp = load_bd(k0 + 1, ohal);
    load_raw(k0 - 1, ok, ro);
    lk[1].kt = (k0 - 2 >= 0) ? kval(Buf<K>::ld(rkz, ok, 0)) : V(0);
    rkt[0] = kval(Buf<K>::ld(rkz, rk, pbk));
    load_raw(k0, rk, rr);
    rbv = Buf<V>::ld(rb, rv, pl(k0) * pbv);
    __syncthreads();

    auto phase = [&](auto QQ, int p) __attribute__((always_inline)) -> bool {
        constexpr int Q = decltype(QQ)::value;
        constexpr int P = Q & 1, QB = (Q + 3) & 3, QT = (Q + 1) & 3, QBB = (Q + 2) & 3;
        const int m = k0 - 1 + p;
        const bool mz = m >= 1 && m <= n - 2;
        // x2 of plane m at the own vertex
        Lk &cw = lk[P];
        widen(ro, lk[P ^ 1].kt, cw);
        V x2m;
        {
            const V(*t1)[XW] = sx1[Q];
            const V xc = t1[ly + 2][lx + 2];
            const V ax = apply7(xc, t1[ly + 2][lx + 1], t1[ly + 2][lx + 3], t1[ly + 1][lx + 2], t1[ly + 3][lx + 2],
                                sx1[QB][ly + 2][lx + 2], sx1[QT][ly + 2][lx + 2], cw.kw, cw.ke, cw.ks, cw.kn, cw.kb,
                                cw.kt, L.s);
            const V v = cheb_step_val(xc, xc, bq[Q], ax, cw.d, c1, c2);
            x2m = (own_inner && mz) ? v : V(0);
        }
        if (p + 1 < np) load_raw(m + 1, ok, ro);
        sx2[Q][ly + 1][lx + 1] = x2m;
        if (m >= k0 && m < k1) Buf<V>::template st<kNT>(x2m, rout, ov, pl(m) * pbv);
        // x2 of plane m on the ring (planes k0 .. kend: the in-plane neighbours of the residual)
        if (p >= 1 && p + 1 < np && ring_wave) {
            Lk w;
            widen(rr, rkt[P ^ 1], w);
            rkt[P] = w.kt;
            const V(*t1)[XW] = sx1[Q];
            const int ry = gy + 1, rx = gx + 1;
            const V xc = t1[ry][rx];
            const V ax = apply7(xc, t1[ry][rx - 1], t1[ry][rx + 1], t1[ry - 1][rx], t1[ry + 1][rx], sx1[QB][ry][rx],
                                sx1[QT][ry][rx], w.kw, w.ke, w.ks, w.kn, w.kb, w.kt, L.s);
            const V v = cheb_step_val(xc, xc, rbv, ax, w.d, c1, c2);
            if (rng) sx2[Q][gy][gx] = rng_inner ? v : V(0);
            if (p + 2 < np) {
                load_raw(m + 1, rk, rr);
                rbv = Buf<V>::ld(rb, rv, pl(m + 1) * pbv);
            }
        }
        // r of plane m-1 at the own vertex, into the z-sum
        if (p >= 2) {
            const int k = m - 1;
            const Lk &pw = lk[P ^ 1];
            const V(*t2)[YW] = sx2[QB];
            const V xc = t2[ly + 1][lx + 1];
            const V r = bq[QB] - apply7(xc, t2[ly + 1][lx], t2[ly + 1][lx + 2], t2[ly][lx + 1], t2[ly + 2][lx + 1],
                                        sx2[QBB][ly + 1][lx + 1], x2m, pw.kw, pw.ke, pw.ks, pw.kn, pw.kb, pw.kt, L.s);
            if (k & 1) {
                if (k > k0)  // closes coarse plane (k-1)/2
                    Buf<V>::template st<kNT>(fmaT(V(0.25), r, acc), rsrc(zs + (long long)((k - 1) >> 1) * plane, kAll),
                                             ov, 0);
                acc = fmaT(V(0.25), r, V(0));  // opens coarse plane (k+1)/2
            } else {
                acc = fmaT(V(0.5), r, acc);
            }
        }
        // x1 of plane m+2 into LDS (own b kept for x2 and r), b, D^-1 of plane m+3
        if (p + 2 <= np) {
            V(*t1)[XW] = sx1[QBB];
            t1[ly + 2][lx + 2] = cheb_first_val(xp.bv, xp.dv, c0);
            if (hal) t1[hy][hx] = cheb_first_val(hp.bv, hp.dv, c0);
            bq[QBB] = xp.bv;
        }
        if (p + 3 <= np) {
            xp = load_bd(m + 3, ovx);
            hp = load_bd(m + 3, ohal);
        }
        __syncthreads();
        return p + 1 == np;
    };
    for (int p = 0;; p += 4) {
        if (phase(std::integral_constant<int, 0>{}, p)) break;
        if (phase(std::integral_constant<int, 1>{}, p + 1)) break;
        if (phase(std::integral_constant<int, 2>{}, p + 2)) break;
        if (phase(std::integral_constant<int, 3>{}, p + 3)) break;
    }
}

// ---------------------------------------------------------------- transfer operators
// Full-weighting restriction b_c = R r, weights (1/4, 1/2, 1/4) per axis,
// summed in one fixed order on every path: z first (the three fine planes of
// a fine column), then x, then y.
template <typename V>
__device__ __forceinline__ V zsum3(V lo, V mid, V hi) {
    V acc = fmaT(V(0.25), lo, V(0));
    acc = fmaT(V(0.5), mid, acc);
    return fmaT(V(0.25), hi, acc);
}
// the in-plane 3 x 3 weighting of z-summed values s around offset base: x, then y
template <typename V>
__device__ __forceinline__ V plane_sum(const V *s, long long base, int pf) {
    const V w[3] = {V(0.25), V(0.5), V(0.25)};
    V accy = V(0);
#pragma unroll
    for (int bb = 0; bb < 3; ++bb) {
        const V *row = s + base + (long long)(bb - 1) * pf;
        V accx = V(0);
#pragma unroll
        for (int a = 0; a < 3; ++a) accx = fmaT(w[a], row[a - 1], accx);
        accy = fmaT(w[bb], accx, accy);
    }
    return accy;
}
// b_c at coarse vertex (I,J,K) from a stored fine residual r (the 27 fine
// vertices of an interior coarse vertex are interior).
template <typename V>
__device__ __forceinline__ V restrict_at(const V *r, int pf, long long plf, int I, int J, int K_) {
    const V w[3] = {V(0.25), V(0.5), V(0.25)};
    V accy = V(0);
    for (int bb = 0; bb < 3; ++bb) {
        V accx = V(0);
        for (int a = 0; a < 3; ++a) {
            const long long o = (long long)(2 * K_) * plf + (long long)(2 * J + bb - 1) * pf + 2 * I + a - 1;
            accx = fmaT(w[a], zsum3(r[o - plf], r[o], r[o + plf]), accx);
        }
        accy = fmaT(w[bb], accx, accy);
    }
    return accy;
}
// (P e) at fine vertex (i,j,k): trilinear, tensor product of the 1D rules
// (even index -> coarse i/2, odd -> mean of (i-1)/2 and (i+1)/2).
template <typename V>
__device__ __forceinline__ V prolong_at(const V *e, int pc, long long plc, int i, int j, int k) {
    const int i0 = i >> 1, i1 = (i + 1) >> 1, j0 = j >> 1, j1 = (j + 1) >> 1, k0 = k >> 1,
              k1 = (k + 1) >> 1;
    const V wi = (i & 1) ? V(0.5) : V(1), wj = (j & 1) ? V(0.5) : V(1), wk = (k & 1) ? V(0.5) : V(1);
    const int ni = (i & 1) ? 2 : 1, nj = (j & 1) ? 2 : 1, nk = (k & 1) ? 2 : 1;
    V accz = V(0);
    for (int c = 0; c < nk; ++c) {
        const int kk = c ? k1 : k0;
        V accy = V(0);
        for (int bb = 0; bb < nj; ++bb) {
            const int jj = bb ? j1 : j0;
            V accx = V(0);
            for (int a = 0; a < ni; ++a) {
                const int ii = a ? i1 : i0;
                accx = fmaT(wi, e[(long long)kk * plc + (long long)jj * pc + ii], accx);
            }
            accy = fmaT(wj, accx, accy);
        }
        accz = fmaT(wk, accy, accz);
    }
    return accz;
}

// b_c = R r for a fine residual r held in memory (Galerkin levels, written by
// the 27-point residual sweep).  One thread per coarse column (I, J) marching
// in K; the order of restrict_at, so both paths round identically.
template <typename V>
__global__ __launch_bounds__(NT) void k_restrict(int nc, int pc, long long plc, Tiling t, int pf, long long plf,
                                                 const V *__restrict__ r, V *__restrict__ bc,
                                                 const int *__restrict__ skip) {
    if (skip && *skip) return;
    const Column c = tile_column(nc, t);
    if (!c.active) return;
    long long oc = (long long)c.k0 * plc + (long long)c.j * pc + c.i;
    for (int K = c.k0; K < c.k1; ++K, oc += plc) bc[oc] = restrict_at(r, pf, plf, c.i, c.j, K);
}

// The residual of a 7-point level reduced along z on the fly: the thread of
// fine column (i, j) computes r = b - A u plane by plane (the arithmetic of
// k_residual) and stores, for each coarse plane K of its chunk, the z-sum
// s(i,j,K) = r(2K-1)/4 + r(2K)/2 + r(2K+1)/4 at s[K * plane + j * pitch + i]
// (fine rows, coarse plane index).  Chunks have an even number of planes and
// start on an odd plane, so a chunk needs one plane beyond its end (its
// neighbour computes that plane too).  Half the fine writes of a stored
// residual, and the restriction that follows reads half as much.
template <typename V, typename K>
__global__ __launch_bounds__(NT) void k_residual_zr(Lev<V, K> L, Tiling t, const V *__restrict__ b,
                                                    const V *__restrict__ u, V *__restrict__ s,
                                                    const int *__restrict__ skip) {
    if (skip && *skip) return;
    const Column c = tile_column(L.n, t);
    if (!c.active) return;
    const int pitch = L.pitch;
    const long long plane = L.plane;
    // N - 1 is even on a level that restricts, so k1 is odd, or N - 1 with
    // N - 2 (odd) the last plane needed: the march always ends on an odd plane
    const int kend = min(c.k1, L.n - 2);
    long long o = (long long)c.k0 * plane + (long long)c.j * pitch + c.i;
    V ub = u[o - plane], up = u[o];
    V kb = kval(L.kz[o - plane]);
    V acc = V(0);
    for (int k = c.k0; k <= kend; ++k, o += plane) {
        const V ut = u[o + plane];
        const V uw = u[o - 1], ue = u[o + 1], us = u[o - pitch], un = u[o + pitch];
        const V kw = kval(L.kx[o - 1]), ke = kval(ldnt(&L.kx[o])), ks = kval(L.ky[o - pitch]),
                kn = kval(L.ky[o]), kt = kval(ldnt(&L.kz[o]));
        const V r = ldnt(&b[o]) - apply7(up, uw, ue, us, un, ub, ut, kw, ke, ks, kn, kb, kt, L.s);
        if (k & 1) {
            if (k > c.k0) {  // closes coarse plane (k-1)/2
                const long long os = (long long)((k - 1) >> 1) * plane + (long long)c.j * pitch + c.i;
                stnt(fmaT(V(0.25), r, acc), &s[os]);
            }
            acc = fmaT(V(0.25), r, V(0));  // opens coarse plane (k+1)/2
        } else {
            acc = fmaT(V(0.5), r, acc);
        }
        ub = up;
        up = ut;
        kb = kt;
    }
}

// b_c = R r from the z-sums of k_residual_zr: the in-plane 3x3 weighting.
template <typename V>
__global__ __launch_bounds__(NT) void k_restrict_xy(int nc, int pc, long long plc, Tiling t, int pf, long long plf,
                                                    const V *__restrict__ s, V *__restrict__ bc,
                                                    const int *__restrict__ skip) {
    if (skip && *skip) return;
    const Column c = tile_column(nc, t);
    if (!c.active) return;
    const long long col = (long long)(2 * c.j) * pf + 2 * c.i;
    long long oc = (long long)c.k0 * plc + (long long)c.j * pc + c.i;
    for (int K = c.k0; K < c.k1; ++K, oc += plc) bc[oc] = plane_sum(s, (long long)K * plf + col, pf);
}

// x += P e by coarse cells: the thread of cell (I,J,K) reads its 8 corner
// values and updates the 8 fine vertices (2I+a, 2J+b, 2K+c), a,b,c in {0,1}.
// Each value is summed in the order of prolong_at (z outer, then y, then x,
// lower coarse index first), so both paths round identically.  Fine vertices
// on the boundary receive combinations of coarse boundary zeros and stay 0.
template <int A, int B, int C, typename V>
__device__ __forceinline__ V cell_val(const V (&e)[2][2][2]) {
    const V wi = A ? V(0.5) : V(1), wj = B ? V(0.5) : V(1), wk = C ? V(0.5) : V(1);
    V accz = V(0);
#pragma unroll
    for (int c = 0; c <= C; ++c) {
        V accy = V(0);
#pragma unroll
        for (int bb = 0; bb <= B; ++bb) {
            V accx = V(0);
#pragma unroll
            for (int a = 0; a <= A; ++a) accx = fmaT(wi, e[c][bb][a], accx);
            accy = fmaT(wj, accx, accy);
        }
        accz = fmaT(wk, accy, accz);
    }
    return accz;
}
template <int B, int C, typename V>
__device__ __forceinline__ void cell_row(V *x, long long o, const V (&e)[2][2][2]) {
    typedef typename Vec2<V>::type V2;
    V2 v = ldnt((const V2 *)(x + o));
    v.x = v.x + cell_val<0, B, C>(e);
    v.y = v.y + cell_val<1, B, C>(e);
    stnt(v, (V2 *)(x + o));
}
template <typename V>
__global__ __launch_bounds__(NT) void k_prolong(int pitch, long long plane, int nc, int pc, long long plc,
                                                const V *__restrict__ e, V *__restrict__ x,
                                                const int *__restrict__ skip) {
    if (skip && *skip) return;
    const int I = blockIdx.x * TX + (threadIdx.x & (TX - 1));
    const int J = blockIdx.y * TY + (threadIdx.x >> 6);
    const int K_ = blockIdx.z;
    if (I > nc - 2 || J > nc - 2) return;
    V ev[2][2][2];
#pragma unroll
    for (int c = 0; c < 2; ++c)
#pragma unroll
        for (int bb = 0; bb < 2; ++bb)
#pragma unroll
            for (int a = 0; a < 2; ++a) ev[c][bb][a] = e[(long long)(K_ + c) * plc + (long long)(J + bb) * pc + I + a];
    const long long o = (long long)(2 * K_) * plane + (long long)(2 * J) * pitch + 2 * I;
    cell_row<0, 0>(x, o, ev);
    cell_row<1, 0>(x, o + pitch, ev);
    cell_row<0, 1>(x, o + plane, ev);
    cell_row<1, 1>(x, o + plane + pitch, ev);
}

// ---------------------------------------------------------------- coarsest solve
// x = (L L^T)^-1 b over the m interior unknowns of the coarsest level, by one
// workgroup: column-oriented forward and backward substitution in FP64.
template <typename V>
__device__ void chol_solve_block(int n, int pitch, long long plane, int m, const double *Lf, const V *b, V *x,
                                 double *y) {
    const int nn = n - 2;
    for (int u = threadIdx.x; u < m; u += blockDim.x) {
        const int i = 1 + u % nn, j = 1 + (u / nn) % nn, k = 1 + u / (nn * nn);
        y[u] = (double)b[(long long)k * plane + (long long)j * pitch + i];
    }
    __syncthreads();
    for (int c = 0; c < m; ++c) {  // L w = b
        const double yc = y[c] / Lf[(long long)c * m + c];
        __syncthreads();
        if (threadIdx.x == 0) y[c] = yc;
        for (int r = c + 1 + threadIdx.x; r < m; r += blockDim.x) y[r] = fmaT(-Lf[(long long)r * m + c], yc, y[r]);
        __syncthreads();
    }
    for (int c = m - 1; c >= 0; --c) {  // L^T y = w
        const double yc = y[c] / Lf[(long long)c * m + c];
        __syncthreads();
        if (threadIdx.x == 0) y[c] = yc;
        for (int r = threadIdx.x; r < c; r += blockDim.x) y[r] = fmaT(-Lf[(long long)c * m + r], yc, y[r]);
        __syncthreads();
    }
    for (int u = threadIdx.x; u < m; u += blockDim.x) {
        const int i = 1 + u % nn, j = 1 + (u / nn) % nn, k = 1 + u / (nn * nn);
        x[(long long)k * plane + (long long)j * pitch + i] = (V)y[u];
    }
    __syncthreads();
}

template <typename V>
__global__ __launch_bounds__(256) void k_coarse_solve(int n, int pitch, long long plane, int m,
                                                      const double *__restrict__ Lf, const V *__restrict__ b,
                                                      V *__restrict__ x, const int *__restrict__ skip) {
    if (skip && *skip) return;
    __shared__ double y[MAX_COARSE];
    chol_solve_block(n, pitch, plane, m, Lf, b, x, y);
}

// ---------------------------------------------------------------- persistent coarse kernel
// Levels s..last-1 of the V-cycle plus the coarsest solve in ONE launch, run
// by a team of one or a few co-resident workgroups: every sweep is a
// team-strided loop over the level's interior vertices followed by a team
// barrier (a workgroup barrier for one workgroup, a device-wide barrier
// otherwise).  Each vertex is computed by exactly one thread with the value
// functions the grid kernels call, so the result does not depend on the team
// size or on the switch level.

// Device-wide barrier of `n` workgroups (cooperative launch guarantees they
// are co-resident).  Generation counting; the wait is bounded: after ~2^24
// polls the barrier records an error and stops waiting (every later barrier
// of the kernel then passes at once), so a kernel always terminates.
struct GridBar {
    unsigned count, gen, err, pad;
};
__device__ void grid_sync(GridBar *gb, unsigned n) {
    __threadfence();  // release this thread's global writes at device scope
    __syncthreads();
    if (threadIdx.x == 0) {
        if (__hip_atomic_load(&gb->err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == 0u) {
            const unsigned g = __hip_atomic_load(&gb->gen, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT);
            const unsigned arrived = __hip_atomic_fetch_add(&gb->count, 1u, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT);
            if (arrived == n - 1) {
                __hip_atomic_store(&gb->count, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                __hip_atomic_fetch_add(&gb->gen, 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
            } else {
                unsigned polls = 0;
                while (__hip_atomic_load(&gb->gen, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT) == g) {
                    __builtin_amdgcn_s_sleep(1);
                    if (++polls > (1u << 24)) {
                        __hip_atomic_store(&gb->err, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                        break;
                    }
                }
            }
        }
    }
    __syncthreads();
    __threadfence();  // acquire: later loads see the other workgroups' writes
}

struct Team {
    int rank, size;  // this workgroup among the active ones
    GridBar *bar;    // null for a single workgroup
    __device__ int first() const { return rank * (int)blockDim.x + (int)threadIdx.x; }
    __device__ int stride() const { return size * (int)blockDim.x; }
    __device__ void sync() const {
        if (size == 1)
            __syncthreads();
        else
            grid_sync(bar, (unsigned)size);
    }
};

__device__ __forceinline__ void vertex_of(int n, int u, int &i, int &j, int &k) {
    const int nn = n - 2;
    i = 1 + u % nn;
    j = 1 + (u / nn) % nn;
    k = 1 + u / (nn * nn);
}

template <typename V, typename K>
__device__ void p_cheb_first(const Team &T, const LevBuf<V, K> &lb, V *out, V c) {
    const Lev<V, K> &L = lb.L;
    const int np = (L.n - 2) * (L.n - 2) * (L.n - 2);
    for (int u = T.first(); u < np; u += T.stride()) {
        int i, j, k;
        vertex_of(L.n, u, i, j, k);
        const long long o = (long long)k * L.plane + (long long)j * L.pitch + i;
        out[o] = cheb_first_val(lb.b[o], L.dinv[o], c);
    }
    T.sync();
}
template <typename V, typename K>
__device__ void p_cheb_step(const Team &T, const LevBuf<V, K> &lb, const V *x, const V *xp, int pm, V *out, V c1,
                            V c2) {
    const Lev<V, K> &L = lb.L;
    const int np = (L.n - 2) * (L.n - 2) * (L.n - 2);
    for (int u = T.first(); u < np; u += T.stride()) {
        int i, j, k;
        vertex_of(L.n, u, i, j, k);
        const long long o = (long long)k * L.plane + (long long)j * L.pitch + i;
        V ax, d, up;
        if (L.a27) {  // uniform over the level
            ax = apply27_at(L.a27, L.nel, x, o, L.pitch, L.plane);
            d = L.a27[(long long)d27(0, 0, 0) * L.nel + o];
            up = x[o];
        } else {
            Nbr<V, K> q;
            load_k(L, o, q);
            load_u(L, x, o, q);
            ax = apply7(q.up, q.uw, q.ue, q.us, q.un, q.ub, q.ut, q.kw, q.ke, q.ks, q.kn, q.kb, q.kt, L.s);
            d = diag7(q.kw, q.ke, q.ks, q.kn, q.kb, q.kt, L.s);
            up = q.up;
        }
        const V diff = pm == 0 ? V(0) : pm == 1 ? up : up - xp[o];
        out[o] = cheb_step_val(up, diff, lb.b[o], ax, d, pm == 0 ? V(0) : c1, c2);
    }
    T.sync();
}
template <typename V>
__device__ void p_copy(const Team &T, int n, int pitch, long long plane, const V *src, V *dst) {
    const int np = (n - 2) * (n - 2) * (n - 2);
    for (int u = T.first(); u < np; u += T.stride()) {
        int i, j, k;
        vertex_of(n, u, i, j, k);
        const long long o = (long long)k * plane + (long long)j * pitch + i;
        dst[o] = src[o];
    }
    T.sync();
}

// Smoothing schedule shared by both paths (see the host-side driver): the
// iterate alternates between x and t1; odd degrees end with a copy into x.
template <typename V, typename K>
__device__ void p_smooth(const Team &T, const LevBuf<V, K> &lb, const ChebCoef<V> &cc, bool from_zero) {
    const Lev<V, K> &L = lb.L;
    V *bufs[2] = {lb.x, lb.t1};
    int cur;  // index of the buffer holding x_j
    int prev; // buffer holding x_{j-1} (or -1)
    if (from_zero) {
        if (cc.m == 1) {
            p_cheb_first(T, lb, lb.x, cc.cfirst);
            return;
        }
        p_cheb_first(T, lb, lb.t1, cc.cfirst);  // x_1 in t1
        cur = 1;
        prev = -1;  // x_0 = 0
    } else {
        p_cheb_step(T, lb, lb.x, (const V *)nullptr, 0, lb.t1, V(0), cc.cfirst);  // x_1 in t1
        cur = 1;
        prev = 0;
        if (cc.m == 1) {
            p_copy(T, L.n, L.pitch, L.plane, lb.t1, lb.x);
            return;
        }
    }
    for (int j = 1; j < cc.m; ++j) {
        const int dst = 1 - cur;  // the buffer of x_{j-1} (or the free one)
        if (prev < 0)
            p_cheb_step(T, lb, bufs[cur], (const V *)nullptr, 1, bufs[dst], cc.c1[j], cc.c2[j]);
        else
            p_cheb_step(T, lb, bufs[cur], bufs[prev], 2, bufs[dst], cc.c1[j], cc.c2[j]);
        prev = cur;
        cur = dst;
    }
    if (cur != 0) p_copy(T, L.n, L.pitch, L.plane, lb.t1, lb.x);
}

// `spread` > 1 packs the team onto one XCD: the launch has nactive*spread
// workgroups and only those with blockIdx % spread == 0 work (dispatch is
// round-robin over the XCDs); the others return at once.
// phase 0: levels s..last-1 down, the coarsest solve on level `last`, and
//          back up (a whole V-cycle below s);
// phase 1: only the down sweep of levels s..last-1 (right-hand side of `last`);
// phase 2: only the up sweep of levels last-1..s (correction from `last`).
// Phases 1 and 2 let a team run the middle levels while a single workgroup
// runs the ones below (multi-stage agglomeration).
// Levels are copied into registers (value copies): stores through the level
// pointers could otherwise alias the level table and force reloads of every
// base pointer after each store.  cc[l]: Chebyshev coefficients of level l.
template <typename V, typename K>
__device__ void persistent_cycle(const Team &T, const LevBuf<V, K> *lv, const ChebCoef<V> *cc, int s, int last,
                                 const double *Lf, int m, int phase, double *y) {
    for (int l = s; l < last && phase != 2; ++l) {
        const LevBuf<V, K> F = lv[l];
        const LevBuf<V, K> C = lv[l + 1];
        p_smooth(T, F, cc[l], true);
        // r = b - A x into t1 (free after smoothing), then full weighting of r
        const int mf = F.L.n - 2, npf = mf * mf * mf;
        for (int u = T.first(); u < npf; u += T.stride()) {
            int i, j, k;
            vertex_of(F.L.n, u, i, j, k);
            const long long o = (long long)k * F.L.plane + (long long)j * F.L.pitch + i;
            F.t1[o] = F.b[o] - apply_at(F.L, F.x, o);
        }
        T.sync();
        const int nc = C.L.n, mc = nc - 2;
        const int np = mc * mc * mc;
        for (int u = T.first(); u < np; u += T.stride()) {
            const int I = 1 + u % mc, J = 1 + (u / mc) % mc, K_ = 1 + u / (mc * mc);
            C.b[(long long)K_ * C.L.plane + (long long)J * C.L.pitch + I] =
                restrict_at(F.t1, F.L.pitch, F.L.plane, I, J, K_);
        }
        T.sync();
    }
    if (phase == 1) return;
    if (phase == 0) {
        if (T.rank == 0) {
            const LevBuf<V, K> C = lv[last];
            chol_solve_block(C.L.n, C.L.pitch, C.L.plane, m, Lf, C.b, C.x, y);
        }
        T.sync();
    }
    for (int l = last - 1; l >= s; --l) {
        const LevBuf<V, K> F = lv[l];
        const LevBuf<V, K> C = lv[l + 1];
        const int mf = F.L.n - 2;
        const int np = mf * mf * mf;
        for (int u = T.first(); u < np; u += T.stride()) {
            const int i = 1 + u % mf, j = 1 + (u / mf) % mf, k = 1 + u / (mf * mf);
            const long long o = (long long)k * F.L.plane + (long long)j * F.L.pitch + i;
            F.x[o] = F.x[o] + prolong_at(C.x, C.L.pitch, C.L.plane, i, j, k);
        }
        T.sync();
        p_smooth(T, F, cc[l], false);
    }
}

template <typename V, typename K>
__global__ __launch_bounds__(NT_PERSIST) void k_persistent(const LevBuf<V, K> *__restrict__ lv,
                                                           const ChebCoef<V> *__restrict__ cc, int s, int last,
                                                           const double *__restrict__ Lf, int m,
                                                           const int *__restrict__ skip, GridBar *bar, int nactive,
                                                           int spread, int phase) {
    if (skip && *skip) return;
    if ((int)blockIdx.x % spread != 0) return;
    const Team T{(int)blockIdx.x / spread, nactive, bar};
    __shared__ double y[MAX_COARSE];
    persistent_cycle(T, lv, cc, s, last, Lf, m, phase, y);
}

// The agglomerated levels held in LDS: one workgroup copies the links, D^-1
// and the right-hand side of level s from HBM into a compact n^3 layout per
// level (pitch n, plane n^2), runs the same cycle on those copies (every
// sweep now reads and writes LDS), and writes the correction x_s back.  Same
// value functions in the same order as the other paths, so the result is
// identical to theirs.  The host launches it only when all levels fit
// (lds_bytes_for below) and only for link (7-point) levels.
__host__ __device__ inline size_t lds_align(size_t b) { return (b + 15) & ~(size_t)15; }
template <typename V, typename K>
__host__ __device__ inline size_t lds_level_bytes(int n) {
    const size_t nv = (size_t)n * n * n;
    return 4 * lds_align(nv * sizeof(V)) + 3 * lds_align(nv * sizeof(K));
}

template <typename V, typename K>
__global__ __launch_bounds__(NT_PERSIST) void k_persistent_lds(const LevBuf<V, K> *__restrict__ lv,
                                                               const ChebCoef<V> *__restrict__ cc, int s, int last,
                                                               const double *__restrict__ Lf, int m,
                                                               const int *__restrict__ skip) {
    if (skip && *skip) return;
    extern __shared__ __align__(16) unsigned char smem[];
    __shared__ LevBuf<V, K> lb[MAX_LEVELS];
    size_t off = 0;
    for (int l = s; l <= last; ++l) {
        const LevBuf<V, K> &G = lv[l];
        const int n = G.L.n;
        const int nv = n * n * n;
        V *x = (V *)(smem + off);
        off += lds_align(nv * sizeof(V));
        V *t1 = (V *)(smem + off);
        off += lds_align(nv * sizeof(V));
        V *b = (V *)(smem + off);
        off += lds_align(nv * sizeof(V));
        V *dv = (V *)(smem + off);
        off += lds_align(nv * sizeof(V));
        K *kx = (K *)(smem + off);
        off += lds_align(nv * sizeof(K));
        K *ky = (K *)(smem + off);
        off += lds_align(nv * sizeof(K));
        K *kz = (K *)(smem + off);
        off += lds_align(nv * sizeof(K));
        if (threadIdx.x == 0) {
            LevBuf<V, K> B = G;
            B.L.pitch = n;
            B.L.plane = (long long)n * n;
            B.L.kx = kx;
            B.L.ky = ky;
            B.L.kz = kz;
            B.L.dinv = dv;
            B.L.a27 = nullptr;
            B.L.nel = nv;
            B.b = b;
            B.x = x;
            B.t1 = t1;
            B.t2 = nullptr;
            lb[l] = B;
        }
        for (int e = threadIdx.x; e < nv; e += blockDim.x) {
            const int i = e % n, j = (e / n) % n, k = e / (n * n);
            const long long g = (long long)k * G.L.plane + (long long)j * G.L.pitch + i;
            kx[e] = G.L.kx[g];
            ky[e] = G.L.ky[g];
            kz[e] = G.L.kz[g];
            dv[e] = G.L.dinv[g];
            b[e] = l == s ? G.b[g] : V(0);
            x[e] = V(0);
            t1[e] = V(0);
        }
    }
    double *y = (double *)(smem + off);
    __syncthreads();
    const Team T{0, 1, nullptr};
    persistent_cycle(T, (const LevBuf<V, K> *)lb, cc, s, last, Lf, m, 0, y);
    const LevBuf<V, K> &G = lv[s];
    const int n = G.L.n, mi = n - 2, np = mi * mi * mi;
    for (int u = threadIdx.x; u < np; u += blockDim.x) {
        const int i = 1 + u % mi, j = 1 + (u / mi) % mi, k = 1 + u / (mi * mi);
        G.x[(long long)k * G.L.plane + (long long)j * G.L.pitch + i] = lb[s].x[(k * n + j) * n + i];
    }
}

// ================================================================ Galerkin coarse operators
// A_c = R A P with trilinear P and R = P^T / 8 (27 coefficients per coarse
// vertex).  Storage: 27 arrays in the level's padded layout, array
// d = (dz+1)*9 + (dy+1)*3 + (dx+1) holds the coefficient of u[p + (dx,dy,dz)];
// boundary vertices and padding hold 0.

// 1D trilinear weight of coarse index offset `c` at fine offset `q` (both
// relative to the coarse vertex, fine offset counted on the fine grid).
__host__ __device__ constexpr double pw1(int q, int c) {
    return (q - 2 * c) == 0 ? 1.0 : ((q - 2 * c) == 1 || (q - 2 * c) == -1) ? 0.5 : 0.0;
}

// One thread per coarse interior vertex I: for every fine point p = 2I + dp
// (dp in -1..1 per axis), every fine neighbour q = p + dq of the fine stencil,
// and every coarse vertex J = I + D, add R[I][p] A[p][q] P[q][J] to a[D].  The
// p and q loops run at run time; the 27 D terms are unrolled so that the sums
// stay in registers (weights that vanish contribute exact zeros).  Fine values
// at boundary q and coarse values at boundary J are excluded (zero Dirichlet
// data).
template <bool LINKS>
__global__ __launch_bounds__(128) void k_galerkin(int n, int pitch, long long plane, const double *__restrict__ kx,
                                                  const double *__restrict__ ky, const double *__restrict__ kz,
                                                  const double *__restrict__ af, long long nel_f, int nc, int pc,
                                                  long long plc, double *__restrict__ ac, long long nel_c) {
    const long long idx = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    const int m = nc - 2;
    if (idx >= (long long)m * m * m) return;
    const int I = 1 + (int)(idx % m), J = 1 + (int)((idx / m) % m), K_ = 1 + (int)(idx / ((long long)m * m));
    const double s = (double)(n - 1) * (double)(n - 1);
    double acc[27];
#pragma unroll
    for (int d = 0; d < 27; ++d) acc[d] = 0.0;
    // coarse vertices off the boundary, per axis and offset -1, 0, 1
    const double ci[3] = {I > 1 ? 1.0 : 0.0, 1.0, I < nc - 2 ? 1.0 : 0.0};
    const double cj[3] = {J > 1 ? 1.0 : 0.0, 1.0, J < nc - 2 ? 1.0 : 0.0};
    const double ck[3] = {K_ > 1 ? 1.0 : 0.0, 1.0, K_ < nc - 2 ? 1.0 : 0.0};
    for (int dp = 0; dp < 27; ++dp) {
        const int px = dp % 3 - 1, py = (dp / 3) % 3 - 1, pz = dp / 9 - 1;
        const int pi = 2 * I + px, pj = 2 * J + py, pk = 2 * K_ + pz;
        const double r = pw1(px, 0) * pw1(py, 0) * pw1(pz, 0) / 8.0;
        const long long po = (long long)pk * plane + (long long)pj * pitch + pi;
        for (int dq = 0; dq < 27; ++dq) {
            const int qx = dq % 3 - 1, qy = (dq / 3) % 3 - 1, qz = dq / 9 - 1;
            const int nz = (qx != 0) + (qy != 0) + (qz != 0);
            if (LINKS && nz > 1) continue;
            const int qi = pi + qx, qj = pj + qy, qk = pk + qz;
            if (qi < 1 || qj < 1 || qk < 1 || qi > n - 2 || qj > n - 2 || qk > n - 2) continue;
            double a;
            if (LINKS) {
                if (nz == 0)
                    a = s * (((kx[po - 1] + kx[po]) + (ky[po - pitch] + ky[po])) + (kz[po - plane] + kz[po]));
                else if (qx)
                    a = -s * kx[qx < 0 ? po - 1 : po];
                else if (qy)
                    a = -s * ky[qy < 0 ? po - pitch : po];
                else
                    a = -s * kz[qz < 0 ? po - plane : po];
            } else {
                a = af[(long long)dq * nel_f + po];
            }
            const double ra = r * a;
            // fine offset of q from 2I on each axis, in -2..2
            const int fx = px + qx, fy = py + qy, fz = pz + qz;
#pragma unroll
            for (int Dz = -1; Dz <= 1; ++Dz)
#pragma unroll
                for (int Dy = -1; Dy <= 1; ++Dy)
#pragma unroll
                    for (int Dx = -1; Dx <= 1; ++Dx) {
                        const double w = pw1(fx, Dx) * pw1(fy, Dy) * pw1(fz, Dz) * ci[Dx + 1] * cj[Dy + 1] *
                                         ck[Dz + 1];
                        acc[d27(Dx, Dy, Dz)] = fmaT(ra, w, acc[d27(Dx, Dy, Dz)]);
                    }
        }
    }
    const long long oc = (long long)K_ * plc + (long long)J * pc + I;
#pragma unroll
    for (int d = 0; d < 27; ++d) ac[(long long)d * nel_c + oc] = acc[d];
}

template <typename V>
__global__ __launch_bounds__(256) void k_cast27(long long n, const double *__restrict__ src, V *__restrict__ dst) {
    const long long stride = (long long)gridDim.x * blockDim.x;
    for (long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += stride) dst[e] = (V)src[e];
}

// D^-1 of a 27-point level: 1 / centre coefficient at interior vertices.
template <typename V>
__global__ __launch_bounds__(NT) void k_dinv27(int n, int pitch, long long plane, Tiling t, const V *__restrict__ a,
                                               long long nel, V *__restrict__ dinv) {
    const Column col = tile_column(n, t);
    if (!col.active) return;
    long long o = (long long)col.k0 * plane + (long long)col.j * pitch + col.i;
    for (int k = col.k0; k < col.k1; ++k, o += plane) dinv[o] = V(1) / a[(long long)d27(0, 0, 0) * nel + o];
}

// 27-point sweeps on Galerkin levels.  MODE 0: y = A u (DOT: partial[wg] =
// sum u.y, the coarse CG's p.Ap);  1: y = b - A u;  2: Chebyshev step (PM as in
// k_cheb_step; the diagonal is the centre coefficient).  out may alias xp.
template <typename V, int MODE, int PM, bool DOT = false>
__global__ __launch_bounds__(NT) void k_sweep27(int n, int pitch, long long plane, Tiling t, const V *__restrict__ a,
                                                long long nel, const V *__restrict__ b, const V *__restrict__ u,
                                                const V *xp, V *out, V c1, V c2, const int *__restrict__ skip,
                                                double *__restrict__ partial = nullptr) {
    if (skip && *skip) return;
    const Column col = tile_column(n, t);
    double dot = 0.0;
    if (col.active) {
        long long o = (long long)col.k0 * plane + (long long)col.j * pitch + col.i;
        for (int k = col.k0; k < col.k1; ++k, o += plane) {
            const V au = apply27_at(a, nel, u, o, pitch, plane);
            if (MODE == 0) {
                out[o] = au;
                if (DOT) dot = fmaT((double)u[o], (double)au, dot);
            } else if (MODE == 1) {
                out[o] = b[o] - au;
            } else {
                const V up = u[o];
                const V d = a[(long long)d27(0, 0, 0) * nel + o];
                const V diff = PM == 0 ? V(0) : PM == 1 ? up : up - xp[o];
                out[o] = cheb_step_val(up, diff, b[o], au, d, PM == 0 ? V(0) : c1, c2);
            }
        }
    }
    if (DOT) {
        const double s = block_sum<NT>(dot);
        if (threadIdx.x == 0) partial[blockIdx.x] = s;
    }
}

// Natural-layout copy of a Galerkin level's stencil: out[v*27 + d], v = (k*n + j)*n + i.
__global__ __launch_bounds__(256) void k_stencil_out(int n, int pitch, long long plane, const double *__restrict__ a,
                                                     long long nel, double *__restrict__ out) {
    const long long v = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= (long long)n * n * n) return;
    const int i = (int)(v % n), j = (int)((v / n) % n), k = (int)(v / ((long long)n * n));
    const long long o = (long long)k * plane + (long long)j * pitch + i;
    for (int d = 0; d < 27; ++d) out[v * 27 + d] = a[(long long)d * nel + o];
}

// ---------------------------------------------------------------- Lanczos on a Galerkin level
// Setup-time estimate of lambda_max(D^-1 A) for the Chebyshev interval of a
// Galerkin level (Lanczos in the D inner product, D = centre coefficients).
// Start vector: 1 + ((7i + 11j + 13k) mod 5) / 4 at interior vertices;
// partial[wg] = its sum of v D v.
__global__ __launch_bounds__(NT) void k_lz_start(int n, int pitch, long long plane, Tiling t,
                                                 const double *__restrict__ a, long long nel,
                                                 double *__restrict__ v, double *__restrict__ partial) {
    const Column col = tile_column(n, t);
    double acc = 0.0;
    if (col.active) {
        long long o = (long long)col.k0 * plane + (long long)col.j * pitch + col.i;
        for (int k = col.k0; k < col.k1; ++k, o += plane) {
            const double u = 1.0 + 0.25 * (double)((7 * col.i + 11 * col.j + 13 * k) % 5);
            v[o] = u;
            acc = fmaT(u * a[(long long)d27(0, 0, 0) * nel + o], u, acc);
        }
    }
    const double sum = block_sum<NT>(acc);
    if (threadIdx.x == 0) partial[blockIdx.x] = sum;
}
// w <- w / d - alpha v - beta vp (w holds A v on entry); partial[wg] = sum w D w
__global__ __launch_bounds__(NT) void k_lz_orth(int n, int pitch, long long plane, Tiling t,
                                                const double *__restrict__ a, long long nel,
                                                const double *__restrict__ v, const double *__restrict__ vp,
                                                double *__restrict__ w, double alpha, double beta,
                                                double *__restrict__ partial) {
    const Column col = tile_column(n, t);
    double acc = 0.0;
    if (col.active) {
        long long o = (long long)col.k0 * plane + (long long)col.j * pitch + col.i;
        for (int k = col.k0; k < col.k1; ++k, o += plane) {
            const double d = a[(long long)d27(0, 0, 0) * nel + o];
            const double wn = w[o] / d - alpha * v[o] - beta * vp[o];
            w[o] = wn;
            acc = fmaT(wn * d, wn, acc);
        }
    }
    const double sum = block_sum<NT>(acc);
    if (threadIdx.x == 0) partial[blockIdx.x] = sum;
}
// v <- v / c at interior vertices
__global__ __launch_bounds__(NT) void k_lz_div(int n, int pitch, long long plane, Tiling t, double *__restrict__ v,
                                               double c) {
    const Column col = tile_column(n, t);
    if (!col.active) return;
    long long o = (long long)col.k0 * plane + (long long)col.j * pitch + col.i;
    for (int k = col.k0; k < col.k1; ++k, o += plane) v[o] = v[o] / c;
}

// ================================================================ PCG vector kernels (FP64)
struct PcgState {
    double bb;      // ||f||^2
    double rho;     // r.z
    double alpha, beta;
    double rr;      // ||r||^2 (recursive)
    double tt;      // ||f - A x||^2 (true)
    double rtol2;   // rtol^2
    int its, max_it;
    int done;       // 1: stop (converged, breakdown or max_it); every loop kernel skips
    int status;     // 0 running/converged, 6 not converged, 7 breakdown
    int restart;    // 1: next p-update uses beta = 0
    int x_pending;  // 1: this iteration's x += alpha p is still to be applied
};

// The PCG vector kernels cover only the interior rows (j, k in 1..n-2) of the
// padded arrays, x index 0 .. 2*half_w-1 in pairs (index 0 and the tail are
// boundary zeros).  No loops: one 16-byte pair per thread, a row split into
// `segs` workgroups of 256 pairs (half_w >= 256), or 256 >> tpr_log2 rows per
// workgroup (short rows).  The workgroup count is fixed by N, so the partial
// sums, and their order, are deterministic.
struct Rows {
    int n, pitch, half_w, tpr_log2, segs, nblocks;
    long long plane;
};
__device__ __forceinline__ bool row_item(const Rows &R, long long &e) {
    const long long nrows = (long long)(R.n - 2) * (R.n - 2);
    long long row;
    int q;
    if (R.segs > 0) {
        row = blockIdx.x / R.segs;
        q = (int)(blockIdx.x % R.segs) * NT_FLAT + (int)threadIdx.x;
    } else {
        row = (long long)blockIdx.x * (NT_FLAT >> R.tpr_log2) + (threadIdx.x >> R.tpr_log2);
        q = threadIdx.x & ((1 << R.tpr_log2) - 1);
    }
    if (row >= nrows || q >= R.half_w) return false;
    e = (1 + row / (R.n - 2)) * R.plane + (1 + row % (R.n - 2)) * (long long)R.pitch + 2 * q;
    return true;
}

// r -= alpha q ; partial = sum r^2 ; MIXED: also b32 = (float) r, the
// right-hand side of the next V-cycle's finest level.
template <typename B>
__global__ __launch_bounds__(NT_FLAT) void k_update_r(Rows R, double *__restrict__ r, const double *__restrict__ q,
                                                      B *__restrict__ b32, const PcgState *__restrict__ st,
                                                      double *__restrict__ partial) {
    if (st->done) return;
    const double a = st->alpha;
    typedef typename Vec2<B>::type B2;
    double acc = 0.0;
    long long e;
    if (row_item(R, e)) {
        double2 rv = ldnt((const double2 *)(r + e));
        const double2 qv = ldnt((const double2 *)(q + e));
        rv.x = fmaT(-a, qv.x, rv.x);
        rv.y = fmaT(-a, qv.y, rv.y);
        stnt(rv, (double2 *)(r + e));
        if (b32) {
            B2 bv;
            bv.x = (B)rv.x;
            bv.y = (B)rv.y;
            stnt(bv, (B2 *)(b32 + e));
        }
        acc = fmaT(rv.x, rv.x, acc);
        acc = fmaT(rv.y, rv.y, acc);
    }
    const double s = block_sum<NT_FLAT>(acc);
    if (threadIdx.x == 0) partial[blockIdx.x] = s;
}

// x += alpha p_old ; p = z + beta p_old (skipped once the loop has stopped,
// when z is stale).  Runs only while this iteration's x update is pending,
// so iterations enqueued after the stop change nothing.  p is FP64 or (MIXED)
// FP32: the new direction is formed in FP64 and rounded once.
template <typename Z, typename PT>
__global__ __launch_bounds__(NT_FLAT) void k_update_xp(Rows R, double *__restrict__ x, PT *__restrict__ p,
                                                       const Z *__restrict__ z, const PcgState *__restrict__ st) {
    if (!st->x_pending) return;
    const double a = st->alpha;
    const bool upd_p = !st->done;
    const double bta = st->beta;
    typedef typename Vec2<Z>::type Z2;
    typedef typename Vec2<PT>::type P2;
    long long e;
    if (row_item(R, e)) {
        const P2 pv = ldnt((const P2 *)(p + e));
        double2 xv = ldnt((const double2 *)(x + e));
        xv.x = fmaT(a, (double)pv.x, xv.x);
        xv.y = fmaT(a, (double)pv.y, xv.y);
        stnt(xv, (double2 *)(x + e));
        if (upd_p) {
            const Z2 zv = ldnt((const Z2 *)(z + e));
            P2 pn;
            pn.x = (PT)fmaT(bta, (double)pv.x, (double)zv.x);
            pn.y = (PT)fmaT(bta, (double)pv.y, (double)zv.y);
            stnt(pn, (P2 *)(p + e));
        }
    }
}

// p = z + beta p   (z FP64 or FP32; p FP64 or, MIXED, FP32)
template <typename Z, typename PT>
__global__ __launch_bounds__(NT_FLAT) void k_update_p(Rows R, PT *__restrict__ p, const Z *__restrict__ z,
                                                      const PcgState *__restrict__ st) {
    if (st->done) return;
    const double bta = st->restart ? 0.0 : st->beta;
    typedef typename Vec2<Z>::type Z2;
    typedef typename Vec2<PT>::type P2;
    long long e;
    if (!row_item(R, e)) return;
    const Z2 zv = *(const Z2 *)(z + e);
    P2 pn;
    if (bta == 0.0) {
        pn.x = (PT)zv.x;
        pn.y = (PT)zv.y;
    } else {
        const P2 pv = *(const P2 *)(p + e);
        pn.x = (PT)fmaT(bta, (double)pv.x, (double)zv.x);
        pn.y = (PT)fmaT(bta, (double)pv.y, (double)zv.y);
    }
    *(P2 *)(p + e) = pn;
}

// partial = sum a.b over the interior rows  (b FP64 or FP32)
template <typename Z>
__global__ __launch_bounds__(NT_FLAT) void k_dot(Rows R, const double *__restrict__ a, const Z *__restrict__ b,
                                                 double *__restrict__ partial, const int *__restrict__ skip) {
    if (skip && *skip) return;
    typedef typename Vec2<Z>::type Z2;
    double acc = 0.0;
    long long e;
    if (row_item(R, e)) {
        const double2 av = *(const double2 *)(a + e);
        const Z2 bv = *(const Z2 *)(b + e);
        acc = fmaT(av.x, (double)bv.x, acc);
        acc = fmaT(av.y, (double)bv.y, acc);
    }
    const double s = block_sum<NT_FLAT>(acc);
    if (threadIdx.x == 0) partial[blockIdx.x] = s;
}

// Plain streaming copy for counter calibration: one 16-byte element per thread.
// Streaming copy of `planes` slabs of n16 16-byte elements each: thread e of
// the grid copies element e of every slab in turn (planes = 1: one element
// per thread; planes > 1: the z-march of the stencil kernels, one slab per
// step), with nontemporal loads and stores.
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
__global__ __launch_bounds__(256) void k_copy_march(long long n16, int planes, const u32x4 *__restrict__ src,
                                                    u32x4 *__restrict__ dst) {
    const long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= n16) return;
    for (int k = 0; k < planes; ++k) {
        const long long o = (long long)k * n16 + e;
        __builtin_nontemporal_store(__builtin_nontemporal_load(&src[o]), &dst[o]);
    }
}

// ---------------------------------------------------------------- inexact coarse CG
// Jacobi-preconditioned CG on the coarsest level of a truncated hierarchy:
// V-precision vectors, FP64 sums, scalars in a PcgState of its own.  Two
// partial arrays (gridDim.x each) carry pairs of sums.
__global__ void k_cg_begin(PcgState *cst, const int *outer_done, double rtol2, int max_it) {
    if (threadIdx.x != 0) return;
    cst->its = 0;
    cst->rtol2 = rtol2;
    cst->max_it = max_it;
    cst->status = 0;
    cst->done = outer_done ? *outer_done : 0;
}
// x = 0, r = b, p = D^-1 r; sums b.b and r.D^-1 r
template <typename V>
__global__ __launch_bounds__(NT_FLAT) void k_cg_start(Rows R, const V *__restrict__ b, V *__restrict__ x,
                                                      V *__restrict__ r, V *__restrict__ p,
                                                      const V *__restrict__ dinv, double *__restrict__ partial,
                                                      const int *__restrict__ skip) {
    if (skip && *skip) return;
    double bb = 0.0, rz = 0.0;
    long long e0;
    if (row_item(R, e0)) {
        for (int t = 0; t < 2; ++t) {
            const long long e = e0 + t;
            const V bv = b[e];
            const V z = bv * dinv[e];
            x[e] = V(0);
            r[e] = bv;
            p[e] = z;
            bb = fmaT((double)bv, (double)bv, bb);
            rz = fmaT((double)bv, (double)z, rz);
        }
    }
    const double s1 = block_sum<NT_FLAT>(bb);
    if (threadIdx.x == 0) partial[blockIdx.x] = s1;
    const double s2 = block_sum<NT_FLAT>(rz);
    if (threadIdx.x == 0) partial[gridDim.x + blockIdx.x] = s2;
}
// x += alpha p, r -= alpha q; sums r.r and r.D^-1 r
template <typename V>
__global__ __launch_bounds__(NT_FLAT) void k_cg_update(Rows R, V *__restrict__ x, V *__restrict__ r,
                                                       const V *__restrict__ p, const V *__restrict__ q,
                                                       const V *__restrict__ dinv, const PcgState *__restrict__ st,
                                                       double *__restrict__ partial) {
    if (st->done) return;
    const V a = (V)st->alpha;
    double rr = 0.0, rz = 0.0;
    long long e0;
    if (row_item(R, e0)) {
        for (int t = 0; t < 2; ++t) {
            const long long e = e0 + t;
            x[e] = fmaT(a, p[e], x[e]);
            const V rv = fmaT(-a, q[e], r[e]);
            r[e] = rv;
            rr = fmaT((double)rv, (double)rv, rr);
            rz = fmaT((double)rv, (double)(rv * dinv[e]), rz);
        }
    }
    const double s1 = block_sum<NT_FLAT>(rr);
    if (threadIdx.x == 0) partial[blockIdx.x] = s1;
    const double s2 = block_sum<NT_FLAT>(rz);
    if (threadIdx.x == 0) partial[gridDim.x + blockIdx.x] = s2;
}
// p = D^-1 r + beta p
template <typename V>
__global__ __launch_bounds__(NT_FLAT) void k_cg_p(Rows R, const V *__restrict__ r, V *__restrict__ p,
                                                  const V *__restrict__ dinv, const PcgState *__restrict__ st) {
    if (st->done) return;
    const V bta = (V)st->beta;
    long long e0;
    if (row_item(R, e0)) {
        for (int t = 0; t < 2; ++t) {
            const long long e = e0 + t;
            p[e] = fmaT(bta, p[e], r[e] * dinv[e]);
        }
    }
}

enum Stage {
    ST_BB = 0, ST_RR0 = 1, ST_RHO0 = 2, ST_ALPHA = 3, ST_RR = 4, ST_BETA = 5, ST_TT = 6,
    ST_BETA_FLEX = 7,  // outer Polak-Ribiere: sums (r.z, q.z)
    ST_C_INIT = 8,     // coarse CG: sums (b.b, r.D^-1 r)
    ST_C_ALPHA = 9,    // coarse CG: p.Ap
    ST_C_RR = 10       // coarse CG: sums (r.r, r.D^-1 r)
};

// Sum `count` partials in a fixed order and advance the PCG state.
constexpr int NT_FIN = 1024;
constexpr int NB_CHUNKS = 256;  // workgroups of the first stage of a large reduction
// First stage of a large reduction: workgroup b sums the contiguous chunk
// [b*chunk, (b+1)*chunk) of p (and, with two, of the second array p + count)
// in a fixed order into out[b] (out[gridDim.x + b]); k_finalize then sums the
// gridDim.x values.  Skipped, like the finalize it feeds, once *skip is set.
__global__ __launch_bounds__(256) void k_reduce_chunks(const double *__restrict__ p, int count, int chunk, int two,
                                                       double *__restrict__ out, const int *__restrict__ skip) {
    if (skip && *skip) return;
    const int lo = blockIdx.x * chunk, hi = min(count, lo + chunk);
    double acc = 0.0, acc2 = 0.0;
    for (int w = lo + (int)threadIdx.x; w < hi; w += 256) {
        acc += p[w];
        if (two) acc2 += p[count + w];
    }
    const double s = block_sum<256>(acc);
    if (threadIdx.x == 0) out[blockIdx.x] = s;
    if (two) {
        const double s2 = block_sum<256>(acc2);
        if (threadIdx.x == 0) out[gridDim.x + blockIdx.x] = s2;
    }
}
// This thread's share of count partial sums (elements threadIdx.x + m*NT_FIN),
// eight loads in flight at a time, added in a fixed order.
__device__ __forceinline__ double fin_thread_sum(const double *__restrict__ p, int count) {
    double acc = 0.0;
    int w = threadIdx.x;
    for (; w + 7 * NT_FIN < count; w += 8 * NT_FIN) {
        double v[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) v[u] = p[w + u * NT_FIN];
        acc += ((v[0] + v[1]) + (v[2] + v[3])) + ((v[4] + v[5]) + (v[6] + v[7]));
    }
    for (; w < count; w += NT_FIN) acc += p[w];
    return acc;
}
__global__ __launch_bounds__(NT_FIN) void k_finalize(const double *__restrict__ partial, int count, int stage,
                                                     PcgState *__restrict__ st) {
    if ((stage == ST_ALPHA || stage == ST_RR || stage == ST_BETA || stage == ST_BETA_FLEX || stage == ST_C_INIT ||
         stage == ST_C_ALPHA || stage == ST_C_RR) &&
        st->done) {
        // an iteration enqueued after the stop: its x update must not run
        if (stage == ST_ALPHA && threadIdx.x == 0) st->x_pending = 0;
        return;
    }
    const bool two = stage == ST_BETA_FLEX || stage == ST_C_INIT || stage == ST_C_RR;
    const double sum = block_sum<NT_FIN>(fin_thread_sum(partial, count));
    const double sum2 = two ? block_sum<NT_FIN>(fin_thread_sum(partial + count, count)) : 0.0;
    if (threadIdx.x != 0) return;
    switch (stage) {
    case ST_BETA_FLEX:  // beta = z_{k+1}.(r_{k+1} - r_k) / rho_k = -alpha (q.z) / rho
        st->beta = -st->alpha * sum2 / st->rho;
        st->rho = sum;
        break;
    case ST_C_INIT:
        st->bb = sum;
        st->rho = sum2;
        if (!(sum > 0.0)) st->done = 1;
        break;
    case ST_C_ALPHA:
        if (!(sum > 0.0) || sum > 1.7e308) {
            st->status = 7;
            st->done = 1;
        } else {
            st->alpha = st->rho / sum;
        }
        break;
    case ST_C_RR:
        st->rr = sum;
        st->its += 1;
        if (!(sum <= st->rtol2 * st->bb) && st->its < st->max_it && sum == sum) {
            st->beta = sum2 / st->rho;
            st->rho = sum2;
        } else {
            st->done = 1;
        }
        break;
    case ST_BB:
        st->bb = sum;
        break;
    case ST_RR0:  // residual of the initial guess
        st->rr = sum;
        if (!(sum == sum) || sum > 1.7e308) {
            st->status = 7;
            st->done = 1;
        } else if (sum <= st->rtol2 * st->bb) {
            st->done = 1;
        }
        break;
    case ST_RHO0:
        st->rho = sum;
        st->restart = 1;
        break;
    case ST_ALPHA:
        if (!(sum > 0.0) || sum > 1.7e308) {  // p.Ap <= 0, NaN or Inf
            st->status = 7;
            st->done = 1;
            st->x_pending = 0;
        } else {
            st->alpha = st->rho / sum;
            st->x_pending = 1;
        }
        break;
    case ST_RR:
        st->rr = sum;
        st->its += 1;
        if (!(sum == sum) || sum > 1.7e308) {
            st->status = 7;
            st->done = 1;
        } else if (sum <= st->rtol2 * st->bb) {
            st->done = 1;
        } else if (st->its >= st->max_it) {
            st->status = 6;
            st->done = 1;
        }
        break;
    case ST_BETA:
        st->beta = sum / st->rho;
        st->rho = sum;
        break;
    case ST_TT:
        st->tt = sum;
        break;
    }
}

// Dense Cholesky factor of the coarsest operator by one workgroup: assemble
// the m x m matrix (m interior unknowns, natural order) from the level's
// links (or its 27 Galerkin coefficients), then factor it in place, right-
// looking: per column, the pivot's square root, the column scaled by it, and
// the trailing lower triangle updated.  Each entry of the trailing block gets
// one update per column, so the parallel order rounds like a serial loop.
// A pivot that is not positive sets st->status = 3 (the operator is not
// positive definite) and the factor is left unusable.  The strict upper
// triangle is zeroed.  m <= MAX_COARSE.
__global__ __launch_bounds__(1024) void k_chol_factor(int n, int pitch, long long plane, const double *__restrict__ kx,
                                                      const double *__restrict__ ky, const double *__restrict__ kz,
                                                      const double *__restrict__ a27, long long nel, double s, int m,
                                                      double *__restrict__ A, PcgState *__restrict__ st) {
    const int nn = n - 2;
    const int tid = (int)threadIdx.x, nth = (int)blockDim.x;
    const long long mm = (long long)m * m;
    for (long long e = tid; e < mm; e += nth) A[e] = 0.0;
    __syncthreads();
    auto unk = [nn](int i, int j, int k) { return ((k - 1) * nn + (j - 1)) * nn + (i - 1); };
    auto in = [n](int i, int j, int k) { return i >= 1 && j >= 1 && k >= 1 && i <= n - 2 && j <= n - 2 && k <= n - 2; };
    for (int p = tid; p < m; p += nth) {  // row p is written by one thread only
        const int i = 1 + p % nn, j = 1 + (p / nn) % nn, k = 1 + p / (nn * nn);
        const long long o = (long long)k * plane + (long long)j * pitch + i;
        double *row = A + (long long)p * m;
        if (a27) {
            for (int d = 0; d < 27; ++d) {
                const int di = d % 3 - 1, dj = (d / 3) % 3 - 1, dk = d / 9 - 1;
                if (in(i + di, j + dj, k + dk)) row[unk(i + di, j + dj, k + dk)] = a27[(long long)d * nel + o];
            }
        } else {
            const double lk[6] = {kx[o - 1], kx[o], ky[o - pitch], ky[o], kz[o - plane], kz[o]};
            const int nb[6][3] = {{i - 1, j, k}, {i + 1, j, k}, {i, j - 1, k}, {i, j + 1, k}, {i, j, k - 1}, {i, j, k + 1}};
            for (int f = 0; f < 6; ++f) {
                row[p] += s * lk[f];
                if (in(nb[f][0], nb[f][1], nb[f][2])) row[unk(nb[f][0], nb[f][1], nb[f][2])] -= s * lk[f];
            }
        }
    }
    __syncthreads();
    __shared__ int bad;
    if (tid == 0) bad = 0;
    for (int col = 0; col < m; ++col) {
        if (tid == 0) {
            const double piv = A[(long long)col * m + col];
            if (!(piv > 0.0)) bad = 1;
            A[(long long)col * m + col] = bad ? 1.0 : sqrt(piv);
        }
        __syncthreads();
        const double piv = A[(long long)col * m + col];
        for (int r = col + 1 + tid; r < m; r += nth) A[(long long)r * m + col] /= piv;
        __syncthreads();
        const int cnt = m - col - 1;
        for (long long e = tid; e < (long long)cnt * cnt; e += nth) {
            const int r = col + 1 + (int)(e / cnt), cc = col + 1 + (int)(e % cnt);
            if (cc <= r)
                A[(long long)r * m + cc] = A[(long long)r * m + cc] - A[(long long)r * m + col] * A[(long long)cc * m + col];
        }
        __syncthreads();
    }
    for (long long e = tid; e < mm; e += nth)
        if (e % m > e / m) A[e] = 0.0;
    if (tid == 0 && bad) st->status = 3;
}

// zero n16 16-byte units (a kernel rather than a memset node: the solve path
// clears its buffers with ordinary launches)
__global__ __launch_bounds__(256) void k_fill_zero(long long n16, uint4 *__restrict__ p) {
    for (long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x; e < n16; e += (long long)gridDim.x * blockDim.x)
        p[e] = make_uint4(0u, 0u, 0u, 0u);
}

// zero a state record (a kernel, not a memset, so the clearing is an ordinary
// launch on the stream)
__global__ void k_clear_state(PcgState *st) {
    if (threadIdx.x == 0) *st = PcgState{};
}

// clear the restart flag after a p-update has consumed it
__global__ void k_clear_restart(PcgState *st) {
    if (threadIdx.x == 0 && !st->done) st->restart = 0;
}

// ================================================================ layout and setup kernels
// natural (N,N,N) FP64 -> padded V; boundary entries written as 0
template <typename V>
__global__ __launch_bounds__(256) void k_to_padded(int n, int pitch, const double *__restrict__ src,
                                                   V *__restrict__ dst) {
    const long long idx = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    const long long tot = (long long)n * n * n;
    if (idx >= tot) return;
    const int i = (int)(idx % n), j = (int)((idx / n) % n), k = (int)(idx / ((long long)n * n));
    const bool in = i >= 1 && j >= 1 && k >= 1 && i <= n - 2 && j <= n - 2 && k <= n - 2;
    dst[((long long)k * n + j) * pitch + i] = in ? (V)src[idx] : V(0);
}
// padded V -> natural FP64 (boundary 0)
template <typename V>
__global__ __launch_bounds__(256) void k_to_natural(int n, int pitch, const V *__restrict__ src,
                                                    double *__restrict__ dst) {
    const long long idx = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    const long long tot = (long long)n * n * n;
    if (idx >= tot) return;
    const int i = (int)(idx % n), j = (int)((idx / n) % n), k = (int)(idx / ((long long)n * n));
    const bool in = i >= 1 && j >= 1 && k >= 1 && i <= n - 2 && j <= n - 2 && k <= n - 2;
    dst[idx] = in ? (double)src[((long long)k * n + j) * pitch + i] : 0.0;
}

// Caller's face arrays (natural shapes, k or ln k) -> padded FP64 level-0
// coefficients.  Active links must be positive and finite; partial[wg] counts
// the violations.  Inactive links are stored as 0.
__global__ __launch_bounds__(256) void k_faces_in(int n, int pitch, const double *__restrict__ kx,
                                                  const double *__restrict__ ky, const double *__restrict__ kz,
                                                  int is_log, double *__restrict__ px, double *__restrict__ py,
                                                  double *__restrict__ pz, double *__restrict__ partial) {
    const long long idx = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    const long long tot = (long long)n * n * n;
    double bad = 0.0;
    if (idx < tot) {
        const int i = (int)(idx % n), j = (int)((idx / n) % n), k = (int)(idx / ((long long)n * n));
        const long long o = ((long long)k * n + j) * pitch + i;
        const bool ij = j >= 1 && j <= n - 2, ik = k >= 1 && k <= n - 2, ii = i >= 1 && i <= n - 2;
        double v;
        // x link (i,i+1): active if j, k interior
        v = 0.0;
        if (i <= n - 2) {
            v = kx[((long long)k * n + j) * (n - 1) + i];
            if (is_log) v = exp(v);
            if (ij && ik) {
                if (!(v > 0.0) || v > 1.7e308) bad += 1.0;
            } else {
                v = 0.0;
            }
        }
        px[o] = v;
        v = 0.0;
        if (j <= n - 2) {
            v = ky[((long long)k * (n - 1) + j) * n + i];
            if (is_log) v = exp(v);
            if (ii && ik) {
                if (!(v > 0.0) || v > 1.7e308) bad += 1.0;
            } else {
                v = 0.0;
            }
        }
        py[o] = v;
        v = 0.0;
        if (k <= n - 2) {
            v = kz[((long long)k * n + j) * n + i];
            if (is_log) v = exp(v);
            if (ii && ij) {
                if (!(v > 0.0) || v > 1.7e308) bad += 1.0;
            } else {
                v = 0.0;
            }
        }
        pz[o] = v;
    }
    const double s = block_sum<256>(bad);
    if (threadIdx.x == 0) partial[blockIdx.x] = s;
}

// Coarse link coefficients from the fine level (both padded FP64): the two
// fine links along the coarse link combine by `rule` (0: (p+q)/2, 1:
// 2pq/(p+q)); the 3x3 lines around it are weighted (1/4,1/2,1/4)^2, summed
// with b (outer) then a (inner) in increasing order.
__device__ __forceinline__ double along_rule(int rule, double p, double q) {
    if (rule == 1) return (p + q) > 0.0 ? 2.0 * p * q / (p + q) : 0.0;
    return 0.5 * (p + q);
}
__global__ __launch_bounds__(256) void k_coarsen(int n, int pitch, long long plane, const double *__restrict__ fx,
                                                 const double *__restrict__ fy, const double *__restrict__ fz, int nc,
                                                 int pc, long long plc, double *__restrict__ cx,
                                                 double *__restrict__ cy, double *__restrict__ cz, int rule) {
    const long long idx = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    const long long tot = (long long)nc * nc * nc;
    if (idx >= tot) return;
    const int I = (int)(idx % nc), J = (int)((idx / nc) % nc), K_ = (int)(idx / ((long long)nc * nc));
    const long long oc = (long long)K_ * plc + (long long)J * pc + I;
    const double w[3] = {0.25, 0.5, 0.25};
    const bool iI = I >= 1 && I <= nc - 2, iJ = J >= 1 && J <= nc - 2, iK = K_ >= 1 && K_ <= nc - 2;
    auto fo = [&](int i, int j, int k) { return (long long)k * plane + (long long)j * pitch + i; };
    double v = 0.0;
    if (I <= nc - 2 && iJ && iK) {
        for (int b = -1; b <= 1; ++b)
            for (int a = -1; a <= 1; ++a)
                v += w[a + 1] * w[b + 1] *
                     along_rule(rule, fx[fo(2 * I, 2 * J + a, 2 * K_ + b)], fx[fo(2 * I + 1, 2 * J + a, 2 * K_ + b)]);
    }
    cx[oc] = v;
    v = 0.0;
    if (J <= nc - 2 && iI && iK) {
        for (int b = -1; b <= 1; ++b)
            for (int a = -1; a <= 1; ++a)
                v += w[a + 1] * w[b + 1] *
                     along_rule(rule, fy[fo(2 * I + a, 2 * J, 2 * K_ + b)], fy[fo(2 * I + a, 2 * J + 1, 2 * K_ + b)]);
    }
    cy[oc] = v;
    v = 0.0;
    if (K_ <= nc - 2 && iI && iJ) {
        for (int b = -1; b <= 1; ++b)
            for (int a = -1; a <= 1; ++a)
                v += w[a + 1] * w[b + 1] *
                     along_rule(rule, fz[fo(2 * I + a, 2 * J + b, 2 * K_)], fz[fo(2 * I + a, 2 * J + b, 2 * K_ + 1)]);
    }
    cz[oc] = v;
}

__global__ __launch_bounds__(256) void k_to_bf16(long long nel, const double *__restrict__ src, bf16 *__restrict__ dst) {
    const long long stride = (long long)gridDim.x * blockDim.x;
    for (long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x; e < nel; e += stride)
        dst[e] = f64_to_bf16_rne(src[e]);
}

// padded level coefficients (any K) -> natural face shapes, FP64
template <typename K>
__global__ __launch_bounds__(256) void k_faces_out(int n, int pitch, const K *__restrict__ px,
                                                   const K *__restrict__ py, const K *__restrict__ pz,
                                                   double *__restrict__ kx, double *__restrict__ ky,
                                                   double *__restrict__ kz) {
    const long long idx = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    const long long tot = (long long)n * n * n;
    if (idx >= tot) return;
    const int i = (int)(idx % n), j = (int)((idx / n) % n), k = (int)(idx / ((long long)n * n));
    const long long o = ((long long)k * n + j) * pitch + i;
    if (i <= n - 2) kx[((long long)k * n + j) * (n - 1) + i] = (double)kval(px[o]);
    if (j <= n - 2) ky[((long long)k * (n - 1) + j) * n + i] = (double)kval(py[o]);
    if (k <= n - 2) kz[((long long)k * n + j) * n + i] = (double)kval(pz[o]);
}

// Adjoint link gradient: for every active link (p,q)
//   g = -h^-2 k (lam_p - lam_q)(phi_p - phi_q)     (= dL/d ln k)
// lam: padded FP64 (boundary 0); phi: caller's natural array (boundary read as 0);
// k: padded FP64 level-0 coefficients.  One thread per vertex p = lower end.
__global__ __launch_bounds__(256) void k_face_gradient(int n, int pitch, double s, const double *__restrict__ lam,
                                                       const double *__restrict__ phi, const double *__restrict__ px,
                                                       const double *__restrict__ py, const double *__restrict__ pz,
                                                       double *__restrict__ gx, double *__restrict__ gy,
                                                       double *__restrict__ gz) {
    const long long idx = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    const long long tot = (long long)n * n * n;
    if (idx >= tot) return;
    const int i = (int)(idx % n), j = (int)((idx / n) % n), k = (int)(idx / ((long long)n * n));
    const long long o = ((long long)k * n + j) * pitch + i;
    auto inner = [&](int a, int b, int c) { return a >= 1 && b >= 1 && c >= 1 && a <= n - 2 && b <= n - 2 && c <= n - 2; };
    const bool pin = inner(i, j, k);
    const double lp = lam[o];
    const double fp = pin ? phi[idx] : 0.0;
    if (i <= n - 2) {
        double g = 0.0;
        const bool qin = inner(i + 1, j, k);
        if (pin || qin) {
            const double fq = qin ? phi[idx + 1] : 0.0;
            g = -s * px[o] * ((lp - lam[o + 1]) * (fp - fq));
        }
        gx[((long long)k * n + j) * (n - 1) + i] = g;
    }
    if (j <= n - 2) {
        double g = 0.0;
        const bool qin = inner(i, j + 1, k);
        if (pin || qin) {
            const double fq = qin ? phi[idx + n] : 0.0;
            g = -s * py[o] * ((lp - lam[o + pitch]) * (fp - fq));
        }
        gy[((long long)k * (n - 1) + j) * n + i] = g;
    }
    if (k <= n - 2) {
        double g = 0.0;
        const bool qin = inner(i, j, k + 1);
        if (pin || qin) {
            const double fq = qin ? phi[idx + (long long)n * n] : 0.0;
            g = -s * pz[o] * ((lp - lam[o + (long long)n * pitch]) * (fp - fq));
        }
        gz[((long long)k * n + j) * n + i] = g;
    }
}

// flat copy / cast between two padded arrays of the same level
template <typename A, typename B>
__global__ __launch_bounds__(NT_FLAT) void k_cast(long long nel, const A *__restrict__ src, B *__restrict__ dst,
                                                  const int *__restrict__ skip) {
    if (skip && *skip) return;
    const long long stride = (long long)gridDim.x * blockDim.x;
    for (long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x; e < nel; e += stride) dst[e] = (B)src[e];
}

}  // namespace gmg
