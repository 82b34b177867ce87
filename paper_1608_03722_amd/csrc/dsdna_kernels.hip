// dsdna_kernels.hip -- gfx950 kernels of one Langevin time step of the
// single-nucleotide dsDNA model (Fosado et al., arXiv:1608.03722).
//
// Per step (all kernels read the step index and the buffer parity from the
// device control block, so a captured graph replays unchanged):
//   k_pairs    excluded volume of the neighbour-list pairs (bead pairs more
//              than LOCAL_BP base pairs apart along the chain), from the FP64
//              bodies, into exact fixed-point sums per bead
//   k_step     one workgroup per tile of TILE_BP base pairs of one replica:
//              stage the tile's FP64 sites in LDS, evaluate every
//              fixed-topology term once into LDS outboxes and the chain-local
//              excluded volume per bead, gather per site (no atomics), add the
//              list pairs' excluded volume, the external loads and the
//              Langevin forces, then integrate the rigid body (FP64) and test
//              whether its bead has moved half the skin since the list was
//              built; its last tile to finish advances the step
//   rebuild    on the steps the host schedules (every K steps): the step
//              kernel bins its new beads (cell, histogram), then k_scan_*
//              (offsets), k_scatter (records into cell order), k_build
//              (neighbour search within the cutoffs plus the skin); k_bin
//              bins a given buffer for a rebuild outside the steps
#include <hip/hip_runtime.h>
#include <math.h>

#include <algorithm>
#include <map>
#include <mutex>
#include <type_traits>
#include <utility>
#include <stdint.h>

#include "dsdna.h"
#include "dsdna_dev.h"

namespace dsdna {

// ------------------------------------------------------------ small vectors

template <typename T>
struct V3 {
    T x, y, z;
};

template <typename T>
__device__ __forceinline__ V3<T> v3(T x, T y, T z) { return V3<T>{x, y, z}; }
template <typename T>
__device__ __forceinline__ V3<T> operator+(V3<T> a, V3<T> b) { return v3(a.x + b.x, a.y + b.y, a.z + b.z); }
template <typename T>
__device__ __forceinline__ V3<T> operator-(V3<T> a, V3<T> b) { return v3(a.x - b.x, a.y - b.y, a.z - b.z); }
template <typename T>
__device__ __forceinline__ V3<T> operator*(V3<T> a, T s) { return v3(a.x * s, a.y * s, a.z * s); }
template <typename T>
__device__ __forceinline__ V3<T> operator-(V3<T> a) { return v3(-a.x, -a.y, -a.z); }
template <typename T>
__device__ __forceinline__ T dot(V3<T> a, V3<T> b) { return a.x * b.x + a.y * b.y + a.z * b.z; }
template <typename T>
__device__ __forceinline__ V3<T> cross(V3<T> a, V3<T> b)
{
    return v3(a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x);
}
template <typename R, typename T>
__device__ __forceinline__ V3<R> cvt(V3<T> a) { return v3((R)a.x, (R)a.y, (R)a.z); }

using D3 = V3<double>;

// Every buffer is global memory, but a pointer read out of the argument block
// is generic to the compiler, which then emits FLAT accesses: 64-bit
// addresses per lane, and each access also counted against the LDS wait
// counter, so that waiting for LDS waits for memory as well.  Accesses in the
// hot kernels go through address-space-1 pointers instead.
// (The host pass, which only parses device code, keeps generic pointers.)
#if defined(__HIP_DEVICE_COMPILE__)
template <typename T>
using gptr = __attribute__((address_space(1))) T *;
#else
template <typename T>
using gptr = T *;
#endif
template <typename T>
__device__ __forceinline__ gptr<T> gmem(T *p) { return (gptr<T>)p; }
// Read-only records that are the same for a whole workgroup (a tile, its
// replica) come through the constant address space: scalar loads.
#if defined(__HIP_DEVICE_COMPILE__)
template <typename T>
using cptr = __attribute__((address_space(4))) const T *;
#else
template <typename T>
using cptr = const T *;
#endif
template <typename T>
__device__ __forceinline__ T cload(const T *p) { return *(cptr<T>)p; }
// Relaxed device-scope atomics on global memory.
template <typename T>
__device__ __forceinline__ T g_add(T *p, T v)
{
    return __hip_atomic_fetch_add(gmem(p), v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
template <typename T>
__device__ __forceinline__ T g_max(T *p, T v)
{
    return __hip_atomic_fetch_max(gmem(p), v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// The body state a step reads was written past the caches by the previous
// step and is read once: loaded non-temporally too (-2 us at 1 Mbp).
__device__ __forceinline__ D3 ld3nt(const double *soa_, int64_t n, int64_t i)
{
    const gptr<const double> soa = gmem(soa_);
    return v3(__builtin_nontemporal_load(soa + i), __builtin_nontemporal_load(soa + n + i),
              __builtin_nontemporal_load(soa + 2 * n + i));
}

__device__ __forceinline__ D3 ld3(const double *soa_, int64_t n, int64_t i)
{
    const gptr<const double> soa = gmem(soa_);
    return v3(soa[i], soa[n + i], soa[2 * n + i]);
}
// The next step's body state is read back only by the next step's tile
// kernel: written past the caches (non-temporal), it leaves the cache to the
// cell-list arrays that the scatter and the excluded-volume pass reuse
// (measured: -2.5 us in the step kernel, -3.8 us in the scatter at 1 Mbp).
__device__ __forceinline__ void st3nt(double *soa_, int64_t n, int64_t i, D3 a)
{
    const gptr<double> soa = gmem(soa_);
    __builtin_nontemporal_store(a.x, soa + i);
    __builtin_nontemporal_store(a.y, soa + n + i);
    __builtin_nontemporal_store(a.z, soa + 2 * n + i);
}

__device__ __forceinline__ void st3(double *soa_, int64_t n, int64_t i, D3 a)
{
    const gptr<double> soa = gmem(soa_);
    soa[i] = a.x;
    soa[n + i] = a.y;
    soa[2 * n + i] = a.z;
}

// Reciprocal and reciprocal square root: the hardware approximations
// (1 ulp) for FP32 forces, correctly rounded division for FP64.
template <typename T>
__device__ __forceinline__ T rcp(T x);
template <>
__device__ __forceinline__ float rcp<float>(float x) { return __builtin_amdgcn_rcpf(x); }
template <>
__device__ __forceinline__ double rcp<double>(double x) { return 1.0 / x; }
// 1/sqrt(x) in FP64 for x > 0: the hardware estimate refined by two Newton
// steps (each doubles the correct bits).
__device__ __forceinline__ double rsq64(double x)
{
    double y = __builtin_amdgcn_rsq(x);
    y = __fma_rn(0.5 * y, __fma_rn(-x * y, y, 1.0), y);
    return __fma_rn(0.5 * y, __fma_rn(-x * y, y, 1.0), y);
}

// 1/x in FP64 for normal x: the hardware estimate refined by two Newton
// steps.
__device__ __forceinline__ double rcp64(double x)
{
    double y = __builtin_amdgcn_rcp(x);
    y = __fma_rn(y, __fma_rn(-x, y, 1.0), y);
    return __fma_rn(y, __fma_rn(-x, y, 1.0), y);
}

// Square root: the hardware approximation in FP32 (forces), exact in FP64.
template <typename T>
__device__ __forceinline__ T fsqrt(T x);
template <>
__device__ __forceinline__ float fsqrt<float>(float x) { return __builtin_amdgcn_sqrtf(x); }
template <>
__device__ __forceinline__ double fsqrt<double>(double x) { return sqrt(x); }
template <typename T>
__device__ __forceinline__ T rsq(T x);
template <>
__device__ __forceinline__ float rsq<float>(float x) { return __builtin_amdgcn_rsqf(x); }
template <>
__device__ __forceinline__ double rsq<double>(double x) { return 1.0 / sqrt(x); }

// Sites of a rigid nucleotide (Sec. 2): bead = R - db u, patch = R + dp u.
// Written with explicit fused multiply-adds so every kernel that recomputes
// a bead position (binning, neighbour search) gets the same bits.
__device__ __forceinline__ D3 bead_of(D3 R, D3 u, double db)
{
    return v3(__fma_rn(-db, u.x, R.x), __fma_rn(-db, u.y, R.y), __fma_rn(-db, u.z, R.z));
}
__device__ __forceinline__ D3 patch_of(D3 R, D3 u, double dp)
{
    return v3(__fma_rn(dp, u.x, R.x), __fma_rn(dp, u.y, R.y), __fma_rn(dp, u.z, R.z));
}

// ------------------------------------------------------------------ Philox

// Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11): ten rounds of two
// 32x32 multiplies per 4-word counter block, key advanced by the Weyl
// increments between rounds.
__device__ __forceinline__ uint4 philox4x32_10(uint4 c, uint2 k)
{
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        if (r) {
            k.x += 0x9E3779B9u;
            k.y += 0xBB67AE85u;
        }
        // one 32 x 32 -> 64-bit product per multiplier
        const uint64_t p0 = (uint64_t)0xD2511F53u * c.x, p1 = (uint64_t)0xCD9E8D57u * c.z;
        const uint32_t lo0 = (uint32_t)p0, hi0 = (uint32_t)(p0 >> 32);
        const uint32_t lo1 = (uint32_t)p1, hi1 = (uint32_t)(p1 >> 32);
        c = make_uint4(hi1 ^ c.y ^ k.x, lo1, hi0 ^ c.w ^ k.y, lo0);
    }
    return c;
}

// The six 32-bit words of nucleotide `id` at `step`: counter
// (id, stream << 16 | call, step lo, step hi), key (seed lo, seed hi);
// words 0..3 of call 0 and 0..1 of call 1.
__device__ __forceinline__ void philox_words(uint64_t seed, uint64_t step, uint32_t id, uint32_t stream,
                                             uint32_t w[6])
{
    const uint2 key = make_uint2((uint32_t)seed, (uint32_t)(seed >> 32));
    const uint4 w0 = philox4x32_10(make_uint4(id, stream << 16, (uint32_t)step, (uint32_t)(step >> 32)), key);
    const uint4 w1 = philox4x32_10(make_uint4(id, (stream << 16) | 1u, (uint32_t)step, (uint32_t)(step >> 32)), key);
    w[0] = w0.x; w[1] = w0.y; w[2] = w0.z; w[3] = w0.w; w[4] = w1.x; w[5] = w1.y;
}

// Six unit-variance numbers (bead xyz, patch xyz): u = (w + 1/2) 2^-32;
// Box-Muller on (w0,w1), (w2,w3), (w4,w5), or sqrt(12)(u - 1/2) for the
// uniform kind.  Evaluated in FP64.
__device__ __forceinline__ void noise6(uint64_t seed, int kind, uint64_t step, uint32_t id, uint32_t stream,
                                       double xi[6])
{
    uint32_t w[6];
    philox_words(seed, step, id, stream, w);
    double u[6];
#pragma unroll
    for (int k = 0; k < 6; ++k) u[k] = ((double)w[k] + 0.5) * 0x1p-32;
    if (kind == 1) {
#pragma unroll
        for (int k = 0; k < 6; ++k) xi[k] = sqrt(12.0) * (u[k] - 0.5);
        return;
    }
#pragma unroll
    for (int k = 0; k < 6; k += 2) {
        const double rad = sqrt(-2.0 * log(u[k]));
        const double ang = 2.0 * M_PI * u[k + 1];
        double s, c;
        sincos(ang, &s, &c);
        xi[k] = rad * c;
        xi[k + 1] = rad * s;
    }
}

// The same numbers evaluated in FP32 (forces in FP32).  For u > 1/2, ln u
// is taken as log1p(-(1 - u)) with 1 - u formed exactly from the integer,
// so the radius keeps its relative accuracy near u = 1; below 1/2 the
// hardware base-2 logarithm is used.  The angle 2 pi u goes to the hardware
// sine and cosine, which take their argument in turns (u itself).
__device__ __forceinline__ void noise6f(uint64_t seed, int kind, uint64_t step, uint32_t id, uint32_t stream,
                                        float xi[6])
{
    uint32_t w[6];
    philox_words(seed, step, id, stream, w);
    if (kind == 1) {
#pragma unroll
        for (int k = 0; k < 6; ++k) {
            // u - 1/2 = (w - 2^31 + 1/2) 2^-32, formed from the signed integer
            const float c = ((float)(int32_t)(w[k] ^ 0x80000000u) + 0.5f) * 0x1p-32f;
            xi[k] = 3.46410161513775459f * c;
        }
        return;
    }
#pragma unroll
    for (int k = 0; k < 6; k += 2) {
        // ln u without a branch.  Below 1/2: the log of u.  From 1/2 up,
        // u = 1 - t with t = (2^32 - 1 - a + 1/2) 2^-32 formed exactly, and
        // ln(1 - t) = log(y) t / (1 - y) for y = 1 - t rounded (Goldberg's
        // log1p identity: exact up to the log's and reciprocal's own
        // errors, 5e-7 relative at worst), -t where y rounds to 1.
        const uint32_t a = w[k];
        const bool up = a >= 0x80000000u;
        const float t = ((float)(up ? ~a : a) + 0.5f) * 0x1p-32f;
        const float y = up ? 1.0f - t : t;
        const float L = __logf(y);
        const float lnu = !up ? L : (y == 1.0f ? -t : L * t * __builtin_amdgcn_rcpf(1.0f - y));
        const float rad = __builtin_amdgcn_sqrtf(-2.0f * lnu);
        const float turns = ((float)w[k + 1] + 0.5f) * 0x1p-32f;
        xi[k] = rad * __builtin_amdgcn_cosf(turns);
        xi[k + 1] = rad * __builtin_amdgcn_sinf(turns);
    }
}

// ------------------------------------------------------------------ errors

__device__ __forceinline__ void raise_error(Ctl *ctl, int code, int64_t step, int64_t id)
{
    if (atomicCAS(&ctl->code, 0, code) == 0) {
        ctl->err_step = step;
        ctl->err_id = id;
    }
}

// Whether the kernels of the positions of step m must not run: an error is
// latched, or the run stops at step m or before (halt_step).
__device__ __forceinline__ bool halted(const Ctl &ctl, int64_t m)
{
    return ctl.code != 0 || (ctl.halt_step != 0 && ctl.halt_step <= m);
}

// --------------------------------------------------------------- cell list

// Cell of a bead and its fixed-point coordinates.  Periodic dims: wrapped
// into [0, L), coordinate = floor(frac * 2^32), cell = floor(coordinate *
// ncell / 2^32) (a function of the coordinate alone, so the neighbour search
// can recompute it from the record); open dims: relative to the replica
// origin, cell = floor(x / h), coordinate = x * 2^24 modulo 2^32.  Returns false if the position is not finite or too
// far from the origin to be binned.
__device__ __forceinline__ int periodic_cell(uint32_t q, int ncell)
{
    return (int)(((uint64_t)q * (uint64_t)(uint32_t)ncell) >> 32);
}

// One dimension of cell_of: cell index and fixed-point coordinate of the
// offset x from the replica origin; ok = false if x cannot be binned.
struct CellDim {
    int c;
    uint32_t q;
    bool ok;
};

__device__ __forceinline__ CellDim cell_dim(const RepInfo &ri, int k, double x)
{
    CellDim r;
    if (ri.flags & (REP_PER_X << k)) {
        double t = x * ri.inv_len[k];
        r.ok = isfinite(t);
        t = r.ok ? t - floor(t) : 0.0;
        r.q = (uint32_t)(uint64_t)(t * 4294967296.0);
        r.c = periodic_cell(r.q, ri.ncell[k]);
    } else {
        r.ok = fabs(x) < 1.0e6;  // also rejects NaN
        const double xs = r.ok ? x : 0.0;
        r.c = (int)floor(xs * ri.inv_h[k]);
        r.q = (uint32_t)(uint64_t)(int64_t)rint(xs * OPEN_QINV);
    }
    return r;
}

__device__ __forceinline__ bool cell_of(const RepInfo &ri, D3 p, int c[3], uint32_t qc[3])
{
    // values, not stores, merge across the branches: the arrays stay in
    // registers
    const CellDim X = cell_dim(ri, 0, p.x - ri.lo[0]), Y = cell_dim(ri, 1, p.y - ri.lo[1]),
                  Z = cell_dim(ri, 2, p.z - ri.lo[2]);
    c[0] = X.c;
    c[1] = Y.c;
    c[2] = Z.c;
    qc[0] = X.q;
    qc[1] = Y.q;
    qc[2] = Z.q;
    return X.ok && Y.ok && Z.ok;
}

__device__ __forceinline__ uint32_t bucket_of(const Grid &g, int cx, int cy, int cz, int rep)
{
    return ((uint32_t)cx + g.A * (uint32_t)cy + g.B * (uint32_t)cz + g.C * (uint32_t)rep) & g.mask;
}

// Tag word of a bead record: strand, steric flag (every third base pair,
// Sec. 2), replica.
__device__ __forceinline__ uint32_t make_tag(int rep, int n, int s)
{
    return (uint32_t)s | ((n % 3) == 0 ? 2u : 0u) | ((uint32_t)rep << 2);
}

// Add n beads to bucket `key` of the histogram and return its previous
// count (16-bit counters, two per word; a bucket past 65535 beads is an
// error, reported for nucleotide i).
__device__ __forceinline__ int hist_add(const StepArgs &a, uint32_t key, int n, int64_t i, int64_t step)
{
    const uint32_t sh = (key & 1u) << 4;
    const uint32_t old = g_add(&a.b.count[key >> 1], (uint32_t)n << sh);
    const int base = (int)((old >> sh) & 0xFFFFu);
    if (base + n > 0xFFFF) raise_error(a.b.ctl, DSDNA_ECELL, step, i);
    return base;
}

// Bin the new bead positions of a tile (all threads of the workgroup call
// this): record, cell and key per bead, then the slots.  The keys of the tile
// are first counted in an LDS hash table (at most WG_THREADS distinct keys in
// WG_THREADS slots, so every probe sequence ends), then one histogram atomic
// per distinct key returns its base slot; a bead's slot is base + its rank
// within the tile.  tab, cnt, base: WG_THREADS entries each of LDS.
__device__ __forceinline__ void bin_tile(const StepArgs &a, uint32_t *tab, uint32_t *cnt, int *base,
                                         const RepInfo &ri, int rep, int n, int s, int64_t i, bool own, D3 bead,
                                         int64_t step)
{
    constexpr uint32_t EMPTY = 0xFFFFFFFFu;  // keys are below 2^28
    const int t = threadIdx.x;
    __syncthreads();
    tab[t] = EMPTY;
    cnt[t] = 0u;
    __syncthreads();
    int e = 0;
    uint32_t rank = 0;
    if (own) {
        int c[3];
        uint32_t qc[3];
        if (!cell_of(ri, bead, c, qc)) {
            raise_error(a.b.ctl, isfinite(bead.x + bead.y + bead.z) ? DSDNA_EDOMAIN : DSDNA_ENAN, step, i);
            c[0] = c[1] = c[2] = 0;
        }
        const uint32_t key = bucket_of(a.g, c[0], c[1], c[2], rep);
        BeadRec r;
        r.x = qc[0];
        r.y = qc[1];
        r.z = qc[2];
        r.tag = make_tag(rep, n, s);
        gmem(a.b.rec)[i] = r;
        if (a.g.any_open) gmem(a.b.rcell)[i] = make_int4(c[0], c[1], c[2], 0);
        gmem(a.b.key)[i] = (int32_t)key;
        e = (int)((key * 2654435761u) >> 24) & (WG_THREADS - 1);
        for (;;) {
            const uint32_t old = atomicCAS(&tab[e], EMPTY, key);
            if (old == EMPTY || old == key) break;
            e = (e + 1) & (WG_THREADS - 1);
        }
        rank = atomicAdd(&cnt[e], 1u);
    }
    __syncthreads();
    if (tab[t] != EMPTY) base[t] = hist_add(a, tab[t], (int)cnt[t], i, step);
    __syncthreads();
    if (own) gmem(a.b.slot)[i] = base[e] + (int)rank;
}

// ------------------------------------------------------------------- tiles

// Work item of workgroup slot b out of n_pad (a multiple of 8): consecutive
// workgroups go to the 8 XCDs in turn, so each XCD is given a contiguous run
// of items (chain neighbours, or neighbouring cells, share an L2).  A
// grid-stride loop over b keeps this when the grid is a multiple of 8.
__device__ __forceinline__ int xcd_item(int b, int n_pad)
{
    const int per = n_pad >> 3;
    return (b & 7) * per + (b >> 3);
}

__device__ __forceinline__ int tile_index(int n_tiles, int n_tiles_pad)
{
    (void)n_tiles;
    return xcd_item((int)blockIdx.x, n_tiles_pad);
}

// ------------------------------------------------------------- tile stage

// The tile's shared arrays, component-major with the site, step or centre
// index fastest, so that the lanes of a wave touch consecutive words (no
// bank conflicts; a [n][3] layout puts 24 or 12 bytes between lanes).
constexpr int TILE_SITES = TILE_NT + 4 * HALO_BP;  // staged sites, halo included
constexpr int TILE_STEPS = 2 * (TILE_BP + 1);      // backbone steps x strands: q = 2 m_i + s
constexpr int TILE_BENDS = 2 * (TILE_BP + 2);      // bending centres x strands: q = 2 m_i + s
template <typename real>
struct TileLds {
    double sB[3][TILE_SITES];              // FP64 bead and patch positions
    double sP[3][TILE_SITES];
    real oStep[4][3][TILE_STEPS];          // per backbone step: bead a, patch a, bead b, patch b
    real oBend[2][3][TILE_BENDS];          // per bending centre: its two end patches
    real oHb[3][TILE_BP];                  // force on strand-0 patch
    uint8_t sOpen[TILE_BP + 2 * HALO_BP];  // open flags of bp n0-2 .. n0+TILE_BP+1
};

template <int N>
__device__ __forceinline__ D3 site3(const double (&a)[3][N], int l) { return v3(a[0][l], a[1][l], a[2][l]); }
template <typename real, int N>
__device__ __forceinline__ V3<real> get_c(const real (&a)[3][N], int q) { return v3(a[0][q], a[1][q], a[2][q]); }
template <typename real, int N>
__device__ __forceinline__ void put_c(real (&a)[3][N], int q, V3<real> v)
{
    a[0][q] = v.x;
    a[1][q] = v.y;
    a[2][q] = v.z;
}

template <typename real>
struct SiteForces {
    V3<real> b, p;
};

__device__ __forceinline__ D3 lds3(const double (*arr)[3], int l) { return v3(arr[l][0], arr[l][1], arr[l][2]); }
template <typename real>
__device__ __forceinline__ void put3(real *dst, V3<real> v)
{
    dst[0] = v.x;
    dst[1] = v.y;
    dst[2] = v.z;
}
template <typename real>
__device__ __forceinline__ V3<real> get3(const real *src) { return v3(src[0], src[1], src[2]); }

constexpr uint32_t ALL_TERMS = (1u << DSDNA_NTERMS) - 1u;
static_assert(WG_THREADS - TILE_NT >= 4 * HALO_BP, "the spare threads of a tile stage its halo");

// Whether the tile slot of base pair bp (relative to the replica start,
// possibly outside it) holds a site: on a ring the two base pairs either
// side of the seam wrap round (bp -2, -1 are nbp-2, nbp-1; bp nbp, nbp+1
// are 0, 1), so every backbone step and bending triple of a tile finds its
// sites in the halo.
// The tile record carries the chain length and the ring flag, so these tests
// need no reload of the replica record.
__device__ __forceinline__ bool site_exists(const Tile &tile, int bp)
{
    return tile.ring ? (bp >= -HALO_BP && bp < tile.n_bp + HALO_BP) : (bp >= 0 && bp < tile.n_bp);
}

// The rigid body a thread loads and stages in LDS (index l <-> bp
// n0 - 2 + l/2, strand l & 1): its own nucleotide for t < TILE_NT, a halo
// site for the next 4 HALO_BP threads, none for the rest.
struct StagedSite {
    int l;         // LDS site index
    bool valid;    // the site exists in the replica
    int64_t i;     // nucleotide index
    D3 R, u;
};

__device__ __forceinline__ StagedSite load_site(const StepArgs &a, const RepInfo &ri, const Tile &tile, int buf)
{
    const int n0 = tile.n0;
    const int t = threadIdx.x;
    StagedSite st;
    st.l = t < TILE_NT ? t + 2 * HALO_BP : (t - TILE_NT < 2 * HALO_BP ? t - TILE_NT : t);
    int bp = n0 - HALO_BP + (st.l >> 1);
    st.valid = st.l < TILE_SITES && site_exists(tile, bp);
    if (tile.ring) bp = bp < 0 ? bp + tile.n_bp : (bp >= tile.n_bp ? bp - tile.n_bp : bp);
    st.i = ri.off + 2 * (int64_t)bp + (st.l & 1);
    st.R = v3(0.0, 0.0, 0.0);
    st.u = st.R;
    if (st.valid) {
        st.R = ld3nt(a.b.R[buf], a.n_nt, st.i);
        st.u = ld3nt(a.b.u[buf], a.n_nt, st.i);
    }
    return st;
}

template <typename real>
__device__ __forceinline__ void stage_site(const StepArgs &a, TileLds<real> &S, const StagedSite &st)
{
    if (!st.valid) return;
    const D3 b = bead_of(st.R, st.u, a.ph.db), p = patch_of(st.R, st.u, a.ph.dp);
    S.sB[0][st.l] = b.x; S.sB[1][st.l] = b.y; S.sB[2][st.l] = b.z;
    S.sP[0][st.l] = p.x; S.sP[1][st.l] = p.y; S.sP[2][st.l] = p.z;
}

// Contact bit of the calling thread's nucleotide in tile tix: its
// excluded-volume accumulator may be nonzero.
__device__ __forceinline__ bool contact_flag(const StepArgs &a, int tix)
{
    const uint32_t w = gmem(a.b.cmask)[(int64_t)tix * CMASK_WORDS + (threadIdx.x >> 5)];
    return (w >> (threadIdx.x & 31)) & 1u;
}

// Excluded-volume force of nucleotide i from the neighbour-list pairs,
// accumulated by k_pairs (only read when its contact bit is set); the entry
// is cleared for the next step.
template <typename real>
__device__ __forceinline__ V3<real> take_fex(const StepArgs &a, int64_t i)
{
    const gptr<longlong4> f = gmem(reinterpret_cast<longlong4 *>(a.b.fex + FEX_WORDS * i));
    const longlong4 hi = f[0];
    const longlong4 lo = f[1];
    if (hi.x | hi.y | hi.z | lo.x | lo.y | lo.z) {
        f[0] = make_longlong4(0, 0, 0, 0);
        f[1] = make_longlong4(0, 0, 0, 0);
    }
    // each part converts exactly; the sum rounds once
    const double sh = 1.0 / FIX_HI, sl = 1.0 / FIX_LO;
    return v3<real>((real)((double)hi.x * sh + (double)lo.x * sl), (real)((double)hi.y * sh + (double)lo.y * sl),
                    (real)((double)hi.z * sh + (double)lo.z * sl));
}

// exp(x) - 1 and atan2(y, x) where the thermal arguments fall: Taylor
// series on |x| < 1/2 (remainder below 6e-9 relative) and for |y| <= x / 4
// (remainder below 1e-10 relative), the library functions elsewhere.
template <typename real>
__device__ __forceinline__ real expm1_small(real x)
{
    if (sizeof(real) == sizeof(double) || !(fabs(x) < (real)0.5)) return expm1(x);
    const real h = x * (real)0.125;
    real p = (real)1 + h;
    p = (real)1 + x * ((real)1 / 7) * p;
    p = (real)1 + x * ((real)1 / 6) * p;
    p = (real)1 + x * (real)0.2 * p;
    p = (real)1 + x * (real)0.25 * p;
    p = (real)1 + x * ((real)1 / 3) * p;
    p = (real)1 + x * (real)0.5 * p;
    return x * p;
}

template <typename real>
__device__ __forceinline__ real atan2_small(real y, real x)
{
    if (sizeof(real) == sizeof(double) || !(fabs(y) <= (real)0.25 * x)) return atan2(y, x);
    const real t = y * rcp(x), t2 = t * t;
    real p = (real)1 / 13;
    p = (real)1 / 11 - t2 * p;
    p = (real)1 / 9 - t2 * p;
    p = (real)1 / 7 - t2 * p;
    p = (real)0.2 - t2 * p;
    p = (real)1 / 3 - t2 * p;
    return t * ((real)1 - t2 * p);
}

// All conservative and external site forces of the calling thread's
// nucleotide, restricted to the terms in `mask`, from the sites every thread
// has staged (stage_site) beforehand; `fex` is the thread's excluded-volume
// force.  Must be called by all threads of the workgroup (it synchronises).
// With energies != nullptr the per-term energies owned by this thread are
// added there (diagnostics only).  DAMP selects the damped dihedral (the
// dihedral_damping reading).
template <typename real, bool DAMP>
__device__ __forceinline__ SiteForces<real> tile_forces(const StepArgs &a, TileLds<real> &S, const RepInfo &ri, const Tile &tile,
                                        V3<real> fex, uint32_t mask, int64_t step, double *energies)
{
    const int t = threadIdx.x;
    const Phys &ph = a.ph;
    const int nbp = tile.n_bp, n0 = tile.n0;
    __syncthreads();
    // every thread has read (and consumed) its accumulator flag before this
    // barrier
    if (t < CMASK_WORDS) gmem(a.b.cmask)[tile_index(a.n_tiles, a.n_tiles_pad) * CMASK_WORDS + t] = 0u;

    // --- hydrogen bonds and open flags (truncated harmonic between the
    //     patches of a base pair, Appendix A)
    const double k2s = ri.k2_scale;
    for (int q = t; q < TILE_BP + 2 * HALO_BP; q += blockDim.x) {
        const int bp = n0 - HALO_BP + q;
        uint8_t open = 0;
        V3<real> f = v3<real>(0, 0, 0);
        if (site_exists(tile, bp)) {
            // the base pair's own K2 multiplier (sequence), if any: a load
            // only when the table is set
            double k2n = k2s;
            if (a.b.k2bp) {
                const int bw = bp < 0 ? bp + nbp : (bp >= nbp ? bp - nbp : bp);
                k2n *= gmem(a.b.k2bp)[ri.off / 2 + bw];
            }
            const D3 d64 = site3(S.sP, 2 * q + 1) - site3(S.sP, 2 * q);
            const double r = sqrt(dot(d64, d64));
            open = r > ph.rc_hb;
            if (!open && (mask & (1u << DSDNA_TERM_HBOND))) {
                const real pref = (real)(ph.hb_pref * k2n);
                real c = (real)2 * pref;
                if (ph.r0_hb != 0.0) c *= (real)1 - (real)(ph.r0_hb / r);  // uniform: no division at r0 = 0
                f = cvt<real>(d64) * c;
                if (energies && q >= HALO_BP && q < TILE_BP + HALO_BP && bp < nbp)
                    energies[DSDNA_TERM_HBOND] += ph.hb_pref * k2n *
                        ((r - ph.r0_hb) * (r - ph.r0_hb) - (ph.rc_hb - ph.r0_hb) * (ph.rc_hb - ph.r0_hb));
            }
        }
        S.sOpen[q] = open;
        if (q >= HALO_BP && q < TILE_BP + HALO_BP) put_c(S.oHb, q - HALO_BP, f);
    }
    // the open flags are read below only under the single-strand rule (the
    // H-bond outboxes are read after the next barrier); the condition is the
    // same for the whole workgroup
    const bool rule = ph.ssdna_rule != 0;
    if (rule) __syncthreads();

    // backbone step m joins bp m and m+1: m = 0 .. nbp-2 on a linear chain,
    // m = -1 .. nbp-1 on a ring (m = -1 and nbp-1 both being the seam step
    // nbp-1 -> 0, seen from either side); a bending triple is centred on bp
    // m = 1 .. nbp-2, or m = -1 .. nbp on a ring
    const bool ring = tile.ring != 0;
    const int step_lo = ring ? -1 : 0, step_hi = ring ? nbp : nbp - 1;
    const int bend_lo = ring ? -1 : 1, bend_hi = ring ? nbp + 1 : nbp - 1;

    // --- backbone steps: FENE + WCA core, Morse, planarity on the pair of
    //     nucleotides (s, m), (s, m+1), m = n0 - 1 + mi
    for (int q = t; q < 2 * (TILE_BP + 1); q += blockDim.x) {
        const int s = q & 1, mi = q >> 1, m = n0 - 1 + mi;
        V3<real> fBa = v3<real>(0, 0, 0), fPa = fBa, fBb = fBa, fPb = fBa;
        if (m >= step_lo && m < step_hi) {
            // LDS site of (s, bp m) and (s, bp m + 1)
            const int la = 2 * (mi + HALO_BP - 1) + s, lb = la + 2;
            const D3 Ba = site3(S.sB, la), Pa = site3(S.sP, la), Bb = site3(S.sB, lb), Pb = site3(S.sP, lb);
            const bool own = mi >= 1;  // step m belongs to the tile that holds nucleotide m
            // backbone: FENE + WCA(eps_bb, sig_bb) between consecutive beads
            if (mask & (1u << DSDNA_TERM_BOND)) {
                const D3 d64 = Bb - Ba;
                const double r2 = dot(d64, d64);
                double x = 1.0 - r2 * ph.inv_R0sq;
                // optional hold of 1 - r^2/R0^2 at 0.1 (fene_clamp); the run
                // stops at R0, or at 2 R0 with the hold
                if (ph.fene_clamp && x < 0.1) x = x <= -3.0 ? 0.0 : 0.1;
                if (x <= 0.0) {
                    raise_error(a.b.ctl, DSDNA_EBOND, step, ri.off + 2 * (int64_t)(m < 0 ? m + nbp : m) + s);
                } else {
                    // FENE attraction and the WCA core cancel to a few percent
                    // near the bond minimum, so (dU/dr)/r is formed in FP64
                    double g = ph.K1 / x;
                    double e = 0.0;
                    if (energies && own) e = -0.5 * ph.K1 * ph.R0 * ph.R0 * log(x);
                    if (r2 < ph.rc_bb * ph.rc_bb) {
                        const double ir2 = 1.0 / r2;
                        const double sr2 = ph.sig_bb * ph.sig_bb * ir2;
                        const double sr6 = sr2 * sr2 * sr2;
                        g -= 24.0 * ph.eps_bb * (2.0 * sr6 * sr6 - sr6) * ir2;
                        if (energies && own) e += 4.0 * ph.eps_bb * (sr6 * sr6 - sr6 + 0.25);
                    }
                    const V3<real> f = cvt<real>(d64 * g);
                    fBa = fBa + f;
                    fBb = fBb - f;
                    if (energies && own) energies[DSDNA_TERM_BOND] += e;
                }
            }
            // stacking: Morse between consecutive patches
            if (mask & (1u << DSDNA_TERM_STACK)) {
                // distance in FP64 and 1 - e^{-x} as -expm1(-x): near the
                // minimum both factors would otherwise cancel in FP32
                // r - r0 = (r^2 - r0^2) / (r + r0) with the numerator in FP64
                const D3 d64 = Pb - Pa;
                const V3<real> d = cvt<real>(d64);
                const double r2_64 = dot(d64, d64);
                const real r = fsqrt((real)r2_64);
                const real dlt = (real)(r2_64 - ph.r0_m * ph.r0_m) * rcp(r + (real)ph.r0_m);
                const real em1 = expm1_small(-(real)ph.lam * dlt);
                const real ir = rcp(r);
                const V3<real> f = d * ((real)(2.0 * ph.K4 * ph.lam) * ((real)1 + em1) * (-em1) * ir);
                fPa = fPa + f;
                fPb = fPb - f;
                if (energies && own) {
                    const double r64 = sqrt(dot(d64, d64)), e64 = exp(-ph.lam * (r64 - ph.r0_m));
                    energies[DSDNA_TERM_STACK] += ph.K4 * (1.0 - e64) * (1.0 - e64);
                }
            }
            // planarity: angle at P_m+1 between P_m and B_m+1, (K5/2)(alpha - a0)^2
            if (mask & (1u << DSDNA_TERM_PLANAR)) {
                // cos and sin of the angle in FP64 (alpha - a0 is small near
                // the minimum), then alpha - a0 as the angle of (cos, sin)
                // rotated by -a0: no cancellation
                const D3 r1d = Pa - Pb, r2d = Bb - Pb;
                const double l11d = dot(r1d, r1d), l22d = dot(r2d, r2d);
                const double ild = rsq64(l11d * l22d);
                double cd = dot(r1d, r2d) * ild;
                cd = cd > 1.0 ? 1.0 : (cd < -1.0 ? -1.0 : cd);
                const double s2 = 1.0 - cd * cd, snd = s2 > 0.0 ? s2 * rsq64(s2) : 0.0;
                const real da = atan2_small((real)(snd * ph.cos_a0 - cd * ph.sin_a0),
                                            (real)(cd * ph.cos_a0 + snd * ph.sin_a0));
                const V3<real> r1 = cvt<real>(r1d), r2 = cvt<real>(r2d);
                const real l11 = (real)l11d, l22 = (real)l22d, il = (real)ild, c = (real)cd, sn = (real)snd;
                const real dUdc = -(real)ph.K5 * da * rcp(sn);
                const V3<real> dca = r2 * il - r1 * (c * rcp(l11)), dcc = r1 * il - r2 * (c * rcp(l22));
                const V3<real> fa = dca * (-dUdc), fc = dcc * (-dUdc);
                fPa = fPa + fa;
                fBb = fBb + fc;
                fPb = fPb - (fa + fc);
                if (energies && own) energies[DSDNA_TERM_PLANAR] += 0.5 * ph.K5 * (double)da * (double)da;
            }
        }
        put_c(S.oStep[0], q, fBa);
        put_c(S.oStep[1], q, fPa);
        put_c(S.oStep[2], q, fBb);
        put_c(S.oStep[3], q, fPb);
    }
    // --- helical twist of the same backbone steps in a pass of its own (its
    //     FP64 intermediates are not live with the other terms'); each
    //     thread adds to the outboxes of the step it wrote above
    for (int q = t; q < 2 * (TILE_BP + 1); q += blockDim.x) {
        const int s = q & 1, mi = q >> 1, m = n0 - 1 + mi;
        if (!(m >= step_lo && m < step_hi)) continue;
        const int la = 2 * (mi + HALO_BP - 1) + s, lb = la + 2;
        const D3 Ba = site3(S.sB, la), Pa = site3(S.sP, la), Bb = site3(S.sB, lb), Pb = site3(S.sP, lb);
        const bool own = mi >= 1;
        const D3 b1d = Pa - Ba, b2d = Pb - Pa, b3d = Bb - Pb;
        V3<real> fBa = v3<real>(0, 0, 0), fPa = fBa, fBb = fBa, fPb = fBa;
        // helical twist: dihedral of (B_m, P_m, P_m+1, B_m+1); gradient as in
        // Blondel & Karplus (1996), free of the 1/sin(phi) singularity
        // open flags of bp m - 1 .. m + 2 (sOpen index of bp m: mi + HALO_BP - 1)
        const uint8_t *op = &S.sOpen[mi + HALO_BP - 2];
        const bool masked = rule && op[1] && op[2] && (op[0] || op[3]);
        if ((mask & (1u << DSDNA_TERM_TWIST)) && !masked) {
            // the angle in FP64: near the minimum sin(phi - d) is a small
            // difference of O(1) products; the gradient directions in the
            // force precision
            const D3 Ad = cross(b1d, b2d), Bd = cross(b2d, b3d);
            const double AAd = dot(Ad, Ad), BBd = dot(Bd, Bd), GGd = dot(b2d, b2d);
            const double iGd = rsq64(GGd), lGd = GGd * iGd;
            const double inv = rsq64(AAd * BBd);
            const double cphi = dot(Ad, Bd) * inv, sphi = lGd * dot(b1d, Bd) * inv;
            // -dU/dphi = K3 sin(phi - d)
            double mdU64 = ph.K3 * (sphi * ph.cos_d - cphi * ph.sin_d);
            D3 dS0 = v3(0.0, 0.0, 0.0), dS1 = dS0, dS2 = dS0, dS3 = dS0;
            double Ud = 0.0, Sd = 1.0;
            if constexpr (DAMP) {
                // dihedral_damping: U sin^3(t1) sin^3(t2) with t1, t2 the bond
                // angles at P_m and P_m+1 (combined bending-torsion form of
                // Bulacu et al., J. Chem. Theory Comput. 9, 3282 (2013)); with c
                // the cosine, d(sin^3)/dc = -3 sin c
                const double L1 = dot(b1d, b1d), L3 = dot(b3d, b3d);
                const double i12 = rsq64(L1 * GGd), i23 = rsq64(GGd * L3);
                const double c1 = dot(b1d, b2d) * i12, c2 = dot(b2d, b3d) * i23;
                const double q1 = fmax(1.0 - c1 * c1, 0.0), q2 = fmax(1.0 - c2 * c2, 0.0);
                const double s1 = sqrt(q1), s2 = sqrt(q2);
                const double S1 = q1 * s1, S2 = q2 * s2;
                const double k1 = -3.0 * s1 * c1, k2 = -3.0 * s2 * c2;
                // gradients of S1 (angle of b1, b2) and S2 (angle of b2, b3)
                const D3 g1u = (b2d * i12 - b1d * (c1 * rcp64(L1))) * k1;
                const D3 g1w = (b1d * i12 - b2d * (c1 * rcp64(GGd))) * k1;
                const D3 g2u = (b3d * i23 - b2d * (c2 * rcp64(GGd))) * k2;
                const D3 g2w = (b2d * i23 - b3d * (c2 * rcp64(L3))) * k2;
                Sd = S1 * S2;
                Ud = ph.K3 * (1.0 + cphi * ph.cos_d + sphi * ph.sin_d);
                dS0 = g1u * (-S2);
                dS1 = (g1u - g1w) * S2 - g2u * S1;
                dS2 = g1w * S2 + (g2u - g2w) * S1;
                dS3 = g2w * S1;
                mdU64 *= Sd;
            }
            const real mdU = (real)mdU64;
            const V3<real> A = cvt<real>(Ad), B = cvt<real>(Bd);
            const real AA = (real)AAd, BB = (real)BBd, iG = (real)iGd, lG = (real)lGd;
            const real FG = (real)dot(b1d, b2d), HG = (real)(-dot(b3d, b2d));
            const real iAA = rcp(AA), iBB = rcp(BB);
            const V3<real> tA = A * (lG * iAA), tB = B * (lG * iBB);
            const V3<real> sA = A * (FG * iAA * iG), sB = B * (HG * iBB * iG);
            fBa = fBa + (-tA) * mdU;
            fPa = fPa + (tA + sA - sB) * mdU;
            fPb = fPb + (-tB - sA + sB) * mdU;
            fBb = fBb + tB * mdU;
            if constexpr (DAMP) {
                fBa = fBa - cvt<real>(dS0 * Ud);
                fPa = fPa - cvt<real>(dS1 * Ud);
                fPb = fPb - cvt<real>(dS2 * Ud);
                fBb = fBb - cvt<real>(dS3 * Ud);
            }
            if (energies && own) energies[DSDNA_TERM_TWIST] += Sd * ph.K3 * (1.0 + cphi * ph.cos_d + sphi * ph.sin_d);
        }
        put_c(S.oStep[0], q, get_c(S.oStep[0], q) + fBa);
        put_c(S.oStep[1], q, get_c(S.oStep[1], q) + fPa);
        put_c(S.oStep[2], q, get_c(S.oStep[2], q) + fBb);
        put_c(S.oStep[3], q, get_c(S.oStep[3], q) + fPb);
    }
    // --- the planarity reading with both triples of a step: the angle at
    //     P_m between P_m+1 and B_m as well, same potential, in a pass of its
    //     own (from the staged sites; each thread adds to the outboxes of
    //     the step it wrote above)
    if (ph.planarity_both && (mask & (1u << DSDNA_TERM_PLANAR))) {
        for (int q = t; q < 2 * (TILE_BP + 1); q += blockDim.x) {
            const int s = q & 1, mi = q >> 1, m = n0 - 1 + mi;
            if (!(m >= step_lo && m < step_hi)) continue;
            const int la = 2 * (mi + HALO_BP - 1) + s, lb = la + 2;
            const D3 Ba = site3(S.sB, la), Pa = site3(S.sP, la), Pb = site3(S.sP, lb);
            const bool own = mi >= 1;
            const D3 q1d = Pb - Pa, q2d = Ba - Pa;
            const double m11d = dot(q1d, q1d), m22d = dot(q2d, q2d);
            const double jld = rsq64(m11d * m22d);
            double ce = dot(q1d, q2d) * jld;
            ce = ce > 1.0 ? 1.0 : (ce < -1.0 ? -1.0 : ce);
            const double t2 = 1.0 - ce * ce, sne = t2 > 0.0 ? t2 * rsq64(t2) : 0.0;
            const real db = atan2_small((real)(sne * ph.cos_a0 - ce * ph.sin_a0), (real)(ce * ph.cos_a0 + sne * ph.sin_a0));
            const V3<real> q1 = cvt<real>(q1d), q2 = cvt<real>(q2d);
            const real jl = (real)jld, cq = (real)ce;
            const real dUde = -(real)ph.K5 * db * rcp((real)sne);
            const V3<real> dqa = q2 * jl - q1 * (cq * rcp((real)m11d)), dqc = q1 * jl - q2 * (cq * rcp((real)m22d));
            const V3<real> ga = dqa * (-dUde), gc = dqc * (-dUde);
            put_c(S.oStep[0], q, get_c(S.oStep[0], q) + gc);
            put_c(S.oStep[1], q, get_c(S.oStep[1], q) - (ga + gc));
            put_c(S.oStep[3], q, get_c(S.oStep[3], q) + ga);
            if (energies && own) energies[DSDNA_TERM_PLANAR] += 0.5 * ph.K5 * (double)db * (double)db;
        }
    }
    // --- Kratky-Porod bending on patches (s, m-1), (s, m), (s, m+1)
    for (int q = t; q < 2 * (TILE_BP + 2); q += blockDim.x) {
        const int s = q & 1, mi = q >> 1, m = n0 - 1 + mi;
        V3<real> f0 = v3<real>(0, 0, 0), f2 = f0;
        // open flags of bp m - 1, m, m + 1
        const uint8_t *op = &S.sOpen[mi + HALO_BP - 2];
        const bool masked = rule && op[0] && op[1] && op[2];
        if ((mask & (1u << DSDNA_TERM_BEND)) && m >= bend_lo && m < bend_hi && !masked) {
            const int la = 2 * (mi + HALO_BP - 2) + s;  // LDS site of (s, bp m - 1)
            const D3 Pa = site3(S.sP, la), Pc = site3(S.sP, la + 2), Pe = site3(S.sP, la + 4);
            const D3 r1 = Pa - Pc, r2 = Pe - Pc;
            const double l11 = dot(r1, r1), l22 = dot(r2, r2), d12 = dot(r1, r2);
            const double il = rsq64(l11 * l22);
            // -dU/dr1 = -K6 il (r2 - r1 (r1.r2) / |r1|^2): the part of r2
            // across r1, a small difference of nearly parallel vectors for a
            // nearly straight triple, so formed in FP64
            const double k = -ph.K6 * il;
            f0 = cvt<real>((r2 - r1 * (d12 * rcp64(l11))) * k);
            f2 = cvt<real>((r1 - r2 * (d12 * rcp64(l22))) * k);
            if (energies && mi >= 1 && mi <= TILE_BP && m < nbp) energies[DSDNA_TERM_BEND] += ph.K6 * (1.0 + d12 * il);
        }
        put_c(S.oBend[0], q, f0);
        put_c(S.oBend[1], q, f2);
    }

    // --- chain-local excluded volume (WCA with the steric/ghost rule of
    //     Sec. 2): the pairs of the thread's own bead with the beads at most
    //     LOCAL_BP base pairs away, every cross-strand bead and, for a steric
    //     bead, the steric beads LOCAL_BP away on its own strand.  Evaluated
    //     from the staged FP64 sites in FP64 (a contact just inside its
    //     cutoff keeps its relative accuracy); each pair is evaluated by the
    //     threads of both its beads, whose results are exact negatives, so
    //     no outbox is needed.  Energies: half of each pair per bead.
    V3<real> floc = v3<real>(0, 0, 0);
    if (t < TILE_NT && n0 + (t >> 1) < nbp && (mask & (1u << DSDNA_TERM_EXCL))) {
        const int s = t & 1, bl = t >> 1, n = n0 + bl;
        const D3 bi = site3(S.sB, t + 2 * HALO_BP);
        D3 acc = v3(0.0, 0.0, 0.0);
        double eh = 0.0;
        auto wca = [&](int lj, double sig2, double rc2) {
            const D3 d = site3(S.sB, lj) - bi;  // from this bead to the other
            const double r2 = dot(d, d);
            if (r2 < rc2) {
                const double ir2 = 1.0 / r2, sr2 = sig2 * ir2, sr6 = sr2 * sr2 * sr2;
                acc = acc - d * (24.0 * ph.eps * (2.0 * sr6 * sr6 - sr6) * ir2);
                if (energies) eh += 2.0 * ph.eps * (sr6 * sr6 - sr6 + 0.25);
            }
        };
        const double sx2 = ph.sig_x * ph.sig_x, rx2 = ph.rc_x * ph.rc_x;
#pragma unroll
        for (int k = -LOCAL_BP; k <= LOCAL_BP; ++k)
            if (site_exists(tile, n + k)) wca(2 * (bl + k + HALO_BP) + (s ^ 1), sx2, rx2);
        if (n % 3 == 0) {  // steric: the steric beads of its strand LOCAL_BP away
            static_assert(LOCAL_BP % 3 == 0, "steric beads are every third base pair");
            const double ss2 = ph.sig_s * ph.sig_s, rs2 = ph.rc_s * ph.rc_s;
            if (site_exists(tile, n - LOCAL_BP)) wca(2 * (bl - LOCAL_BP + HALO_BP) + s, ss2, rs2);
            if (site_exists(tile, n + LOCAL_BP)) wca(2 * (bl + LOCAL_BP + HALO_BP) + s, ss2, rs2);
        }
        floc = cvt<real>(acc);
        if (energies) energies[DSDNA_TERM_EXCL] += eh;
    }
    __syncthreads();

    // --- gather per site (fixed order, no atomics); threads past the tile
    //     own no nucleotide
    const int s = t & 1, bl = t >> 1;
    const int n = t < TILE_NT ? n0 + bl : nbp;
    SiteForces<real> out;
    out.b = v3<real>(0, 0, 0);
    out.p = out.b;
    if (n < nbp) {
        out.b = get_c(S.oStep[2], 2 * bl + s) + get_c(S.oStep[0], 2 * (bl + 1) + s);
        // middle patch of a bending triple: minus the sum of the end forces
        const V3<real> mid = -(get_c(S.oBend[0], 2 * (bl + 1) + s) + get_c(S.oBend[1], 2 * (bl + 1) + s));
        out.p = get_c(S.oStep[3], 2 * bl + s) + get_c(S.oStep[1], 2 * (bl + 1) + s) + get_c(S.oBend[1], 2 * bl + s) +
                mid + get_c(S.oBend[0], 2 * (bl + 2) + s);
        const V3<real> hb = get_c(S.oHb, bl);
        out.p = s == 0 ? out.p + hb : out.p - hb;
    }

    // --- excluded volume: the chain-local pairs above plus the neighbour-list
    //     pairs, accumulated per bead beforehand
    if (n < nbp && (mask & (1u << DSDNA_TERM_EXCL))) {
        out.b = out.b + floc + fex;
        if (energies) energies[DSDNA_TERM_EXCL] += a.b.eex[ri.off + 2 * (int64_t)n + s];
    }
    if (n >= nbp) return out;

    const int l = t + 2 * HALO_BP;
    const D3 bi = site3(S.sB, l);
    const int64_t i = ri.off + 2 * (int64_t)n + s;

    // --- external loads (Sec. 4)
    if (mask & (1u << DSDNA_TERM_EXT)) {
        if (ri.flags & REP_TETHER) {
            const double dz = bi.z - ri.wall_z;
            if (dz <= 0.0) {
                raise_error(a.b.ctl, DSDNA_EWALL, step, i);
            } else if (dz < ph.rc_s) {
                const real z = (real)dz;
                const real iz2 = rcp(z * z);
                const real sr2 = (real)(ph.sig_s * ph.sig_s) * iz2;
                const real sr6 = sr2 * sr2 * sr2;
                out.b.z += (real)(24.0 * ph.eps) * ((real)2 * sr6 * sr6 - sr6) * rcp(z);
                if (energies) {
                    const double s2 = ph.sig_s * ph.sig_s / (dz * dz), s6 = s2 * s2 * s2;
                    energies[DSDNA_TERM_EXT] += 4.0 * ph.eps * (s6 * s6 - s6 + 0.25);
                }
            }
        }
        if (n == nbp - 1) {
            if (ri.flags & REP_PULL)
                out.p = out.p + v3<real>((real)(0.5 * ri.pull[0]), (real)(0.5 * ri.pull[1]), (real)(0.5 * ri.pull[2]));
            if (ri.flags & REP_TORQUE) {
                // couple on the two beads about their midpoint
                const D3 b0 = site3(S.sB, l - s), b1 = site3(S.sB, l - s + 1);
                const D3 cmid = (b0 + b1) * 0.5;
                const D3 G = v3(ri.torque[0], ri.torque[1], ri.torque[2]);
                const double G2 = dot(G, G);
                const D3 Gh = G * (1.0 / sqrt(G2));
                const D3 d0 = b0 - cmid, d1 = b1 - cmid;
                const D3 p0 = d0 - Gh * dot(d0, Gh), p1 = d1 - Gh * dot(d1, Gh);
                const double D = dot(p0, p0) + dot(p1, p1);
                if (D > 0.0) out.b = out.b + cvt<real>(cross(G, s == 0 ? d0 : d1) * (1.0 / D));
            }
        }
    }
    return out;
}


// Rotation of the axis of a free linear rotor by th about unit k:
// u cos th + (k x u) sin th + k (k.u)(1 - cos th).  For th < 1/4 (angular
// speeds below 50 per unit time at dt = 0.005, far in the tail of the
// thermal distribution) cos and sin come from their Taylor series through
// th^16 and th^17, whose remainders are below 1e-25; otherwise sincos.
__device__ __forceinline__ D3 rotate(D3 u, D3 k, double th)
{
    double sn, cs;
    if (th < 0.25) {
        const double t2 = th * th;
        double c = 1.0 / 20922789888000.0;            // 1/16!
        double s = 1.0 / 355687428096000.0;           // 1/17!
        c = 1.0 / 87178291200.0 - t2 * c;             // 1/14!
        s = 1.0 / 1307674368000.0 - t2 * s;           // 1/15!
        c = 1.0 / 479001600.0 - t2 * c;               // 1/12!
        s = 1.0 / 6227020800.0 - t2 * s;              // 1/13!
        c = 1.0 / 3628800.0 - t2 * c;                 // 1/10!
        s = 1.0 / 39916800.0 - t2 * s;                // 1/11!
        c = 1.0 / 40320.0 - t2 * c;                   // 1/8!
        s = 1.0 / 362880.0 - t2 * s;                  // 1/9!
        c = 1.0 / 720.0 - t2 * c;
        s = 1.0 / 5040.0 - t2 * s;
        c = 1.0 / 24.0 - t2 * c;
        s = 1.0 / 120.0 - t2 * s;
        c = 0.5 - t2 * c;
        s = 1.0 / 6.0 - t2 * s;
        cs = 1.0 - t2 * c;
        sn = th * (1.0 - t2 * s);
    } else {
        sincos(th, &sn, &cs);
    }
    return u * cs + cross(k, u) * sn + k * (dot(k, u) * (1.0 - cs));
}

// ---------------------------------------------------------------- k_step

template <typename real, bool DAMP>
__global__ void __launch_bounds__(WG_THREADS, 5) k_step(const StepArgs *__restrict__ A, int mode, int write_full,
                                                       int rebuild_after, int age)
{
    __shared__ TileLds<real> S;
    __shared__ float s_v2[WG_THREADS / 64];
    const StepArgs &a = *A;
    // the loads of a starting workgroup are issued ahead of the arithmetic
    // of the workgroups already in their force phase on the same SIMDs
    // (wave priority, lowered again before the staging): measured 4% faster
    // at 1 Mbp
    __builtin_amdgcn_s_setprio(1);
    const Ctl ctl = cload(a.b.ctl);
    if (halted(ctl, ctl.step)) return;
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        a.b.ctl->done_step = ctl.step;
        a.b.ctl->done_par = ctl.par;
    }
    const int tix = tile_index(a.n_tiles, a.n_tiles_pad);
    if (tix >= a.n_tiles) return;
    const Tile tile = cload(&a.b.tiles[tix]);
    const RepInfo &ri = a.b.rep[tile.rep];
    const int cur = ctl.par, nxt = cur ^ 1;
    const int64_t step = ctl.step;
    const int64_t N = a.n_nt;
    const Phys &ph = a.ph;

    // every global load of this thread up front: its body (or halo site),
    // velocities and excluded-volume force
    const StagedSite site = load_site(a, ri, tile, cur);
    const int s = threadIdx.x & 1;
    const int n = threadIdx.x < TILE_NT ? tile.n0 + (int)(threadIdx.x >> 1) : tile.n_bp;
    const bool own = n < tile.n_bp;
    const int64_t i = site.i;
    D3 R = site.R, u = site.u;
    V3<real> fexv = v3<real>(0, 0, 0);
    const bool flagged = mode != MODE_FROM_FORCES && contact_flag(a, tix);
    if (own && flagged) fexv = take_fex<real>(a, i);
    const bool frozen = (ri.flags & REP_TETHER) && n == 0;
    const bool langevin = own && !frozen && ph.gamma > 0.0 && mode != MODE_FROM_FORCES;
    SiteForces<real> f;
    f.b = v3<real>(0, 0, 0);
    f.p = f.b;
    __builtin_amdgcn_s_setprio(0);
    if (mode != MODE_FROM_FORCES) {
        stage_site(a, S, site);
        f = tile_forces<real, DAMP>(a, S, ri, tile, fexv, ALL_TERMS, step, nullptr);
    }
    // velocities and noise only now: they are not live through the force
    // phase, and the noise is drawn while the velocity loads are in flight
    D3 V = v3(0.0, 0.0, 0.0), L = V;
    BeadRec ref = {0u, 0u, 0u, 0u};  // the bead's record when the list was built
    if (own) {
        V = ld3nt(a.b.V[cur], N, i);
        L = ld3nt(a.b.L[cur], N, i);
        ref = gmem(a.b.rec)[i];
    }
    real xi[6] = {0, 0, 0, 0, 0, 0};
    if (langevin) {
        if (sizeof(real) == sizeof(double)) {
            double x64[6];
            noise6(ph.seed, ph.noise_kind, (uint64_t)step, (uint32_t)i, 0u, x64);
            for (int k = 0; k < 6; ++k) xi[k] = (real)x64[k];
        } else {
            float x32[6];
            noise6f(ph.seed, ph.noise_kind, (uint64_t)step, (uint32_t)i, 0u, x32);
            for (int k = 0; k < 6; ++k) xi[k] = (real)x32[k];
        }
    }
    D3 bead_new = v3(0.0, 0.0, 0.0);
    if (own) {
        D3 fb, fp;  // total site forces of this step
        if (mode == MODE_FROM_FORCES) {
            fb = ld3(a.b.Fb, N, i);
            fp = ld3(a.b.Fp, N, i);
        } else {
            V3<real> lb = v3<real>(0, 0, 0), lp = lb;
            if (langevin) {
                // Langevin forces (Appendix A) per site: friction on the site's
                // velocity on the rigid body plus counter-based noise
                const D3 w = L * ph.inv_I;
                const D3 vb = V + cross(w, u * (-ph.db)), vp = V + cross(w, u * ph.dp);
                if (sizeof(real) == sizeof(double)) {
                    lb = cvt<real>(vb * (-ph.gamma) + v3((double)xi[0], (double)xi[1], (double)xi[2]) * ph.noise_amp);
                    lp = cvt<real>(vp * (-ph.gamma) + v3((double)xi[3], (double)xi[4], (double)xi[5]) * ph.noise_amp);
                } else {
                    const real amp = (real)ph.noise_amp;
                    lb = cvt<real>(vb * (-ph.gamma)) + v3<real>(xi[0], xi[1], xi[2]) * amp;
                    lp = cvt<real>(vp * (-ph.gamma)) + v3<real>(xi[3], xi[4], xi[5]) * amp;
                }
            }
            fb = cvt<double>(f.b + lb);
            fp = cvt<double>(f.p + lp);
        }

        if (frozen) {
            V = v3(0.0, 0.0, 0.0);
            L = V;
            if (write_full) {
                st3(a.b.Vf, N, i, V);
                st3(a.b.Lf, N, i, L);
                st3(a.b.Fb, N, i, fb);
                st3(a.b.Fp, N, i, fp);
                if (a.b.Rf) {
                    st3(a.b.Rf, N, i, R);
                    st3(a.b.uf, N, i, u);
                }
            }
        } else {
            const D3 F = fb + fp;
            const D3 tau = cross(u, fp * ph.dp - fb * ph.db);
            const double km = ph.kick_M;
            if (mode == MODE_NORMAL) {  // second half kick of the previous step
                V = V + F * km;
                L = L + tau * ph.kick;
            }
            if (write_full) {
                st3(a.b.Vf, N, i, V);
                st3(a.b.Lf, N, i, L);
                st3(a.b.Fb, N, i, fb);
                st3(a.b.Fp, N, i, fp);
                if (a.b.Rf) {  // bound arrays: the full-step positions and axes too
                    st3(a.b.Rf, N, i, R);
                    st3(a.b.uf, N, i, u);
                }
            }
            // first half kick, drift, free rotation of the linear rotor
            V = V + F * km;
            L = L + tau * ph.kick;
            R = R + V * ph.dt;
            const D3 w = L * ph.inv_I;
            const double w2 = dot(w, w);
            if (w2 > 0.0) {
                // 1/|w| from the hardware estimate refined by two Newton
                // steps (each doubles the correct bits), then the unit axis
                // and |w| dt from it
                double ri = __builtin_amdgcn_rsq(w2);
                ri = __fma_rn(0.5 * ri, __fma_rn(-w2 * ri, ri, 1.0), ri);
                ri = __fma_rn(0.5 * ri, __fma_rn(-w2 * ri, ri, 1.0), ri);
                u = rotate(u, w * ri, w2 * ri * ph.dt);
            }
            // renormalise: |u|^2 = 1 up to rounding, so one Newton step from 1
            // gives 1/|u| to double precision
            u = u * (1.5 - 0.5 * dot(u, u));
            L = L - u * dot(L, u);
        }
        st3nt(a.b.R[nxt], N, i, R);
        st3nt(a.b.u[nxt], N, i, u);
        st3nt(a.b.V[nxt], N, i, V);
        st3nt(a.b.L[nxt], N, i, L);
        if (!(isfinite(R.x + R.y + R.z) && isfinite(u.x + u.y + u.z))) raise_error(a.b.ctl, DSDNA_ENAN, step + 1, i);
        bead_new = bead_of(R, u, ph.db);
    }
    // --- the neighbour list stays valid while no bead has moved half the
    //     skin since it was built: compare the new bead with its record (the
    //     wrapped fixed-point difference is the exact displacement).  Unless a
    //     rebuild follows this step, a bead that far stops the run at the new
    //     positions.  On the step a rebuild follows, the largest squared
    //     displacement over the interval is kept for the host's schedule.
    bool far = false;
    float v2 = 0.0f;
    (void)age;
    if (own) {
        int c[3];
        uint32_t q[3];
        if (!cell_of(ri, bead_new, c, q))
            raise_error(a.b.ctl, isfinite(bead_new.x + bead_new.y + bead_new.z) ? DSDNA_EDOMAIN : DSDNA_ENAN, step + 1, i);
        const float dx = (float)(int32_t)(q[0] - ref.x) * ri.qlen[0];
        const float dy = (float)(int32_t)(q[1] - ref.y) * ri.qlen[1];
        const float dz = (float)(int32_t)(q[2] - ref.z) * ri.qlen[2];
        const float d2 = dx * dx + dy * dy + dz * dz;
        far = !rebuild_after && d2 >= ph.half_skin2;
        v2 = rebuild_after ? d2 : 0.0f;
    }
    const uint64_t far_lanes = __ballot(far);
    const unsigned lane = threadIdx.x & 63;
    if (far_lanes && lane == (unsigned)__builtin_ctzll(far_lanes))
        g_max((unsigned long long *)&a.b.ctl->halt_step, (unsigned long long)(step + 1));
    // the tile's largest displacement into its own slot (no other tile
    // touches it)
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) v2 = fmaxf(v2, __shfl_xor(v2, d, 64));
    if (lane == 0) s_v2[threadIdx.x >> 6] = v2;
    __syncthreads();
    if (rebuild_after && threadIdx.x == 0) {
        float m = s_v2[0];
        for (int w = 1; w < WG_THREADS / 64; ++w) m = fmaxf(m, s_v2[w]);
        if (m > gmem(a.b.vmax)[tix]) gmem(a.b.vmax)[tix] = m;
    }
    // --- a rebuild follows: bin the new bead (record, cell, key, slot and
    //     histogram), the counting sort's count phase; the force phase's
    //     outboxes hold the binning table
    if (rebuild_after) {
        uint32_t *lds = reinterpret_cast<uint32_t *>(&S.oStep[0][0][0]);
        bin_tile(a, lds, lds + WG_THREADS, reinterpret_cast<int *>(lds + 2 * WG_THREADS), ri, tile.rep, n, s, i,
                 own, bead_new, step + 1);
    }
}

// ------------------------------------------------- neighbour-list rebuild

// Workgroups of the rebuild kernels (grid-stride loops).
constexpr int REBUILD_GRID = 2048;

// Counting-sort count phase: bins the beads of buffer `which` (-1: the
// positions the last step kernel wrote).
// Each bead's record becomes the reference position of the displacement test.
__global__ void __launch_bounds__(WG_THREADS) k_bin(const StepArgs *__restrict__ A, int which)
{
    const StepArgs &a = *A;
    const Ctl ctl = cload(a.b.ctl);
    // which < 0: the positions the last step kernel wrote
    const int64_t step = which < 0 ? ctl.done_step + 1 : ctl.step;
    if (halted(ctl, step)) return;
    __shared__ uint32_t tab[WG_THREADS], cnt[WG_THREADS];
    __shared__ int base[WG_THREADS];
    const int buf = which < 0 ? (ctl.done_par ^ 1) : which;
    const int t = threadIdx.x;
    for (int b = blockIdx.x; b < a.n_tiles_pad; b += gridDim.x) {
        const int tix = xcd_item(b, a.n_tiles_pad);
        if (tix >= a.n_tiles) continue;  // the same for the whole workgroup
        const Tile tile = cload(&a.b.tiles[tix]);
        const RepInfo &ri = a.b.rep[tile.rep];
        const int s = t & 1, n = t < TILE_NT ? tile.n0 + (t >> 1) : tile.n_bp;
        const bool own = n < tile.n_bp;
        const int64_t i = ri.off + 2 * (int64_t)n + s;
        D3 bead = v3(0.0, 0.0, 0.0);
        if (own) bead = bead_of(ld3(a.b.R[buf], a.n_nt, i), ld3(a.b.u[buf], a.n_nt, i), a.ph.db);
        bin_tile(a, tab, cnt, base, ri, tile.rep, n, s, i, own, bead, step);
    }
}

// ------------------------------------------------------- excluded volume

// Excluded-volume sums of the neighbour-list pairs are exact and order
// independent: every contact force component is split into a coarse integer
// number of 1/FIX_HI units and a remainder of 1/FIX_LO units, summed as two
// 64-bit integers, so a bead's total depends neither on which thread
// evaluated a pair nor on the order.

// The two integer parts of force component f (units 2^-8 and 2^-40): v = f
// 2^40 is exact, h the nearest multiple of 2^32 to it, and v - h 2^32 exact
// (the two lie within a factor 2 of each other, or h is 0), then rounded to
// the 2^-40 grid.
__device__ __forceinline__ void fix_split(double f, long long &hi, long long &lo)
{
    const double v = f * FIX_LO;
    const double h = rint(v * (1.0 / 4294967296.0));
    hi = (long long)h;
    lo = __double2ll_rn(v - h * 4294967296.0);
}

// Add the force f (sign +1 or -1) to nucleotide j and set its contact bit
// (bit 2 (n - n0) + s of its tile's mask, the tile thread that owns it).
__device__ __forceinline__ void fex_add(const StepArgs &a, const RepInfo &ri, int64_t j, const long long hi[3],
                                        const long long lo[3], long long sign)
{
    unsigned long long *f = a.b.fex + FEX_WORDS * j;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        if (hi[k]) atomicAdd(f + k, (unsigned long long)(sign * hi[k]));
        if (lo[k]) atomicAdd(f + 4 + k, (unsigned long long)(sign * lo[k]));
    }
    const int64_t jj = j - ri.off;
    const int tb = (int)(jj >> 1) / TILE_BP;
    const int lt = (int)(jj - 2 * (int64_t)TILE_BP * tb);
    atomicOr(&a.b.cmask[(int64_t)(ri.tile0 + tb) * CMASK_WORDS + (lt >> 5)], 1u << (lt & 31));
}

// Excluded volume (WCA, Sec. 2 and App. A) of the neighbour-list pairs, the
// bead pairs more than LOCAL_BP base pairs apart: one thread per pair.  The
// distance is formed from the FP64 bodies of both nucleotides (minimum image
// along periodic edges) and the force in FP64, whatever the precision of the
// other terms: contacts are rare, and near the cutoff the force is a small
// difference of O(1) numbers.  Pairs beyond the cutoff (within the skin)
// contribute nothing.
__global__ void __launch_bounds__(256) k_pairs(const StepArgs *__restrict__ A, int which, int energy, int mode)
{
    const StepArgs &a = *A;
    Ctl *ctl = a.b.ctl;
    const Ctl c0 = *ctl;
    if (c0.code != 0) return;
    int64_t m = c0.step;
    int buf = which < 0 ? c0.par : which;
    if (mode != PAIRS_DIAG) {
        // the first kernel of a step: publish its step and buffer
        m = c0.done_step + 1;
        buf = c0.done_par ^ 1;
        if (blockIdx.x == 0 && threadIdx.x == 0) {
            ctl->step = m;
            ctl->par = buf;
        }
        if (mode == PAIRS_PUBLISH) return;
    }
    if (halted(c0, m)) return;
    const int64_t n = min((int64_t)c0.list_n, a.list_cap);
    const double *Rc = a.b.R[buf], *uc = a.b.u[buf];
    const int64_t N = a.n_nt;
    const Phys &ph = a.ph;
    int64_t bad = -1;
    for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < n; k += (int64_t)gridDim.x * blockDim.x) {
        const PairRec pr = a.b.plist[k];
        const RepInfo &ri = a.b.rep[pr.rep];
        D3 d = bead_of(ld3(Rc, N, pr.j), ld3(uc, N, pr.j), ph.db) - bead_of(ld3(Rc, N, pr.i), ld3(uc, N, pr.i), ph.db);
        if (ri.flags & REP_PER_X) d.x = __fma_rn(-ri.len[0], rint(d.x * ri.inv_len[0]), d.x);
        if (ri.flags & REP_PER_Y) d.y = __fma_rn(-ri.len[1], rint(d.y * ri.inv_len[1]), d.y);
        if (ri.flags & REP_PER_Z) d.z = __fma_rn(-ri.len[2], rint(d.z * ri.inv_len[2]), d.z);
        const double r2 = dot(d, d);
        const double rc = pr.same ? ph.rc_s : ph.rc_x, sig = pr.same ? ph.sig_s : ph.sig_x;
        if (!(r2 < rc * rc)) continue;
        const double ir2 = 1.0 / r2, sr2 = sig * sig * ir2, sr6 = sr2 * sr2 * sr2;
        // force on j (+), on i (-): repulsive
        const D3 f = d * (24.0 * ph.eps * (2.0 * sr6 * sr6 - sr6) * ir2);
        if (!(fabs(f.x) + fabs(f.y) + fabs(f.z) < PAIR_FORCE_MAX)) {
            bad = pr.i;
            continue;
        }
        long long hi[3], lo[3];
        fix_split(f.x, hi[0], lo[0]);
        fix_split(f.y, hi[1], lo[1]);
        fix_split(f.z, hi[2], lo[2]);
        fex_add(a, ri, pr.j, hi, lo, 1);
        fex_add(a, ri, pr.i, hi, lo, -1);
        if (energy) {
            const double eh = 2.0 * ph.eps * (sr6 * sr6 - sr6 + 0.25);  // half the pair energy
            atomicAdd(&a.b.eex[pr.i], eh);
            atomicAdd(&a.b.eex[pr.j], eh);
        }
    }
    if (bad >= 0) raise_error(ctl, DSDNA_ENAN, m, bad);
}

// A bead of the sorted cell list as the neighbour search sees it.
struct ExclBead {
    BeadRec me;
    uint32_t rep, mt, accept;
    const RepInfo *ri;
    bool px, py, pz;
    int c[3];       // its cell
    uint32_t kown;  // its bucket
};

template <bool any_open>
__device__ __forceinline__ ExclBead excl_bead(const StepArgs &a, const BeadRec *__restrict__ srec,
                                              const int4 *__restrict__ scell, int p)
{
    ExclBead B;
    B.me = srec[p];
    B.rep = B.me.tag >> 2;
    B.mt = B.me.tag & 3u;
    // partner types (bit 0 strand, bit 1 steric) this bead interacts with:
    // the other strand always, its own strand steric-steric only
    B.accept = (B.mt & 1u ? 0x5u : 0xAu) | (B.mt & 2u ? (B.mt & 1u ? 0x8u : 0x4u) : 0u);
    B.ri = &a.b.rep[B.rep];
    B.px = B.ri->flags & REP_PER_X;
    B.py = B.ri->flags & REP_PER_Y;
    B.pz = B.ri->flags & REP_PER_Z;
    // any_open: some replica has an open edge; cells were stored by the
    // binning.  Otherwise they follow from the periodic coordinates.
    if (any_open) {
        const int4 cc = scell[p];
        B.c[0] = cc.x;
        B.c[1] = cc.y;
        B.c[2] = cc.z;
    } else {
        B.c[0] = periodic_cell(B.me.x, B.ri->ncell[0]);
        B.c[1] = periodic_cell(B.me.y, B.ri->ncell[1]);
        B.c[2] = periodic_cell(B.me.z, B.ri->ncell[2]);
    }
    B.kown = bucket_of(a.g, B.c[0], B.c[1], B.c[2], (int)B.rep);
    return B;
}

// Does a ghost bead (cross-strand partners only, within rc of it) need the
// neighbour cells below / above it along dimension k?  Periodic dims: from
// its position inside the cell (the low 32 bits of q * ncell); open dims:
// always.
__device__ __forceinline__ void ghost_reach(const RepInfo &ri, int k, uint32_t q, double rc, bool &lo, bool &hi)
{
    if (!(ri.flags & (REP_PER_X << k))) {
        lo = hi = true;
        return;
    }
    const uint64_t frac = (uint64_t)(uint32_t)((uint64_t)q * (uint64_t)(uint32_t)ri.ncell[k]);
    // rc in fractions of the cell, in 2^-32 units (the cell is wider than rc)
    const uint64_t T = (uint64_t)(rc * (double)ri.ncell[k] * ri.inv_len[k] * 4294967296.0);
    lo = frac < T;
    hi = 4294967296ull - frac < T;
}

// Whether nucleotides i and j of replica ri form a chain-local pair (base
// pairs at most LOCAL_BP apart, cyclically on a ring): those pairs are the
// step kernel's.
__device__ __forceinline__ bool local_pair(const RepInfo &ri, int64_t i, int64_t j)
{
    int d = abs((int)((i - ri.off) >> 1) - (int)((j - ri.off) >> 1));
    if (ri.flags & REP_RING) d = min(d, ri.n_bp - d);
    return d <= LOCAL_BP;
}

// Neighbour-list build (Verlet list with a skin) from the key-sorted cell
// list: one thread per sorted record, so the lanes of a wave hold beads of
// neighbouring cells and read overlapping candidate ranges.  A bead pairs
// with every bead of the other strand and, if steric, with the steric beads
// of its own strand (Sec. 2); a pair enters the list when its distance is
// below its WCA cutoff plus the skin and it is not chain-local.  Each pair is
// found once (half stencil): the thread of a bead scans the later records of
// its own bucket, the next cell of its row, the row above (dy = +1) and the
// three rows of the next layer (dz = +1), as one stream of five record
// ranges.  A ghost bead has only cross-strand partners, so it skips the
// neighbour cells farther than that reach from its position (exact: a
// skipped cell holds no bead that close).  The candidate counts of a
// workgroup's records vary a lot, so the records are handed to the threads
// in order of decreasing count (a counting sort in LDS) and each wave's lanes
// carry similar loads.  Distances come from the fixed-point records (exact
// differences; the list cutoffs carry a slack for their FP32 evaluation).
constexpr int EXCL_THREADS = 256;  // records per workgroup (sorted by load together)

// (8 waves per SIMD: the search is latency-bound, and 64 VGPRs cost a few
// spilled registers; measured faster at 1 Mbp than 6 waves at 72-75 VGPRs)
template <bool any_open>
__global__ void __launch_bounds__(EXCL_THREADS, 8) k_build(const StepArgs *__restrict__ A, const BeadRec *__restrict__ srec,
                                              const int *__restrict__ sid, const int4 *__restrict__ scell,
                                              const int *__restrict__ start)
{
    const StepArgs &a = *A;
    Ctl *ctl = a.b.ctl;
    const int64_t built_step = ctl->done_step + 1;  // the positions k_bin binned
    if (halted(*ctl, built_step)) return;
    const int t = threadIdx.x;
    // the histogram has served this cell list: clear it for the next
    // binning (streaming stores while this kernel is bound by its search)
    {
        int4 *c4 = reinterpret_cast<int4 *>(a.b.count);
        const int n4 = a.g.nbucket >> 3, stride = (int)(gridDim.x * blockDim.x);
        for (int k = (int)(blockIdx.x * blockDim.x + threadIdx.x); k < n4; k += stride) c4[k] = make_int4(0, 0, 0, 0);
    }
    if (blockIdx.x == 0 && t == 0) ctl->rebuilds += 1;
    const Phys &ph = a.ph;
    const float rcs2 = (float)ph.rl2_s, rcx2 = (float)ph.rl2_x;
    const uint32_t cap = (uint32_t)min(a.list_cap, (int64_t)0x7FFFFFFF);

    __shared__ int s_sh[5][EXCL_THREADS];
    __shared__ int s_pre[5][EXCL_THREADS];
    __shared__ uint32_t s_pk[EXCL_THREADS];
    __shared__ int s_tot[EXCL_THREADS];
    __shared__ uint16_t s_wr[EXCL_THREADS];
    __shared__ int s_hist[64];
    __shared__ int s_order[EXCL_THREADS];
    const int nblk = (int)((a.n_nt + EXCL_THREADS - 1) / EXCL_THREADS);
    const int nblk_pad = (nblk + 7) / 8 * 8;
    for (int vb = blockIdx.x; vb < nblk_pad; vb += gridDim.x) {
    const int blk = xcd_item(vb, nblk_pad);
    const int p0 = blk * EXCL_THREADS;
    __syncthreads();  // the LDS of the previous block is free

    // --- the candidate stream of record p0 + t: stream position k of range
    // q sits at k + s_sh[q] in the sorted records; s_pre[q] = first stream
    // position of range q.  Range 0: the rest of the own bucket and the next
    // cell; ranges 1..4: rows (dy, dz) = (+1, 0), (-1, +1), (0, +1), (+1, +1)
    // over the needed dx.  At a periodic x face the neighbour cell across
    // the face is not next to the others in bucket order: the range keeps
    // the contiguous cells and that one cell is walked later (bit 8 + q of
    // s_wr).  A range whose buckets would wrap past the end of the bucket
    // array (rare) is empty here and walked cell by cell (bit q).
    int key = 0;
    {
        int total = 0;
        uint32_t wrapped = 0, pk = 0;
        if (p0 + t < a.n_nt) {
            const int p = p0 + t;
            const ExclBead B = excl_bead<any_open>(a, srec, scell, p);
            const RepInfo &ri = *B.ri;
            const int ncx = ri.ncell[0], ncy = ri.ncell[1], ncz = ri.ncell[2];
            auto wrap = [&](int v, int n, bool per_) { return per_ ? (v < 0 ? v + n : (v >= n ? v - n : v)) : v; };
            bool xm = true, xp = true, ym = true, yp = true, zm = true, zp = true;
            if (!(B.mt & 2u)) {
                const double rc = ph.rc_x + ph.skin + 1e-3;
                ghost_reach(ri, 0, B.me.x, rc, xm, xp);
                ghost_reach(ri, 1, B.me.y, rc, ym, yp);
                ghost_reach(ri, 2, B.me.z, rc, zm, zp);
            }
#pragma unroll
            for (int q = 0; q < 5; ++q) {
                int l0 = 0, h0 = 0;
                bool wr = false;
                // the cells cx + dlo .. cx + dhi are contiguous buckets; a
                // neighbour across a periodic x face is walked separately
                const bool face_lo = B.px && B.c[0] == 0 && xm, face_hi = B.px && B.c[0] == ncx - 1 && xp;
                const int dlo = (xm && !face_lo) ? -1 : 0, dhi = (xp && !face_hi) ? 1 : 0;
                bool face = false;
                if (q == 0) {
                    face = face_hi;
                    wr = dhi > 0 && B.kown == a.g.mask;
                    l0 = p + 1;
                    h0 = wr ? p + 1 : start[B.kown + dhi + 1];
                } else {
                    const int dy = q == 1 ? 1 : q - 3, dz = q == 1 ? 0 : 1;
                    const bool need = (dy > 0 ? yp : (dy < 0 ? ym : true)) && (dz == 0 || zp);
                    if (need) {
                        const int cy = wrap(B.c[1] + dy, ncy, B.py), cz = wrap(B.c[2] + dz, ncz, B.pz);
                        const uint32_t kc = bucket_of(a.g, B.c[0], cy, cz, (int)B.rep);
                        face = face_lo || face_hi;
                        wr = (dlo < 0 && kc == 0u) || (dhi > 0 && kc == a.g.mask);
                        l0 = wr ? 0 : start[(int)kc + dlo];
                        h0 = wr ? 0 : start[(int)kc + dhi + 1];
                    }
                }
                wrapped |= ((uint32_t)wr << q) | ((uint32_t)(face && !wr) << (8 + q));
                s_pre[q][t] = total;
                s_sh[q][t] = l0 - total;
                if (q >= 1) pk |= (uint32_t)min(total, 127) << (8 * (q - 1));
                total += h0 - l0;
            }
            // the dx reach (a ghost's) for the cell-by-cell walk
            wrapped |= (xm ? 0x20u : 0u) | (xp ? 0x40u : 0u);
            (void)zm;
        }
        s_pk[t] = pk;
        s_tot[t] = total;
        s_wr[t] = (uint16_t)wrapped;
        // (clamped: every key is a histogram bin, so s_order below is always a
        // full permutation of the workgroup's threads)
        key = min(max(total >> 1, 0), 63);
    }

    // --- counting sort of the workgroup's records by decreasing count
    if (t < 64) s_hist[t] = 0;
    __syncthreads();
    const int rank = atomicAdd(&s_hist[63 - key], 1);
    __syncthreads();
    if (t < 64) {
        const int v = s_hist[t];
        int x = v;
#pragma unroll
        for (int d = 1; d < 64; d <<= 1) {
            const int o = __shfl_up(x, d, 64);
            if (t >= d) x += o;
        }
        s_hist[t] = x - v;
    }
    __syncthreads();
    s_order[s_hist[63 - key] + rank] = t;
    __syncthreads();
    const int src = s_order[t];
    const int p = p0 + src;
    if (p < a.n_nt) {

    // --- the candidates of record p (its stream is LDS column src)
    const ExclBead B = excl_bead<any_open>(a, srec, scell, p);
    const BeadRec me = B.me;
    const uint32_t rep = B.rep, mt = B.mt, accept = B.accept;
    const RepInfo &ri = *B.ri;
    const int64_t i = sid[p];
    const float qx = ri.qlen[0], qy = ri.qlen[1], qz = ri.qlen[2];
    const bool px = B.px, py = B.py, pz = B.pz;
    const bool open_any = any_open && !(px && py && pz);
    const int *c = B.c;

    // list test of candidate o: every test evaluated, no branch.  (A
    // candidate is never the bead itself: its own bucket is searched from
    // the next record on, and the host keeps the 27 cells around any cell in
    // distinct buckets.)  FAST: one replica (no record of another replica
    // shares a bucket) and the same fixed-point unit along x, y and z, so the
    // squared distance is compared in those units.
    const float rcs2u = rcs2 / (qx * qx), rcx2u = rcx2 / (qx * qx);
    auto test = [&](const BeadRec &o, auto fast) -> bool {
        const uint32_t ot = o.tag & 3u;
        const bool same = ((ot ^ mt) & 1u) == 0u;
        const float dx = (float)(int32_t)(o.x - me.x);
        const float dy = (float)(int32_t)(o.y - me.y);
        const float dz = (float)(int32_t)(o.z - me.z);
        if constexpr (decltype(fast)::value) {
            const float r2u = dx * dx + dy * dy + dz * dz;
            return (r2u < (same ? rcs2u : rcx2u)) & (((accept >> ot) & 1u) != 0u);
        } else {
            const float ex = dx * qx, ey = dy * qy, ez = dz * qz;
            const float r2f = ex * ex + ey * ey + ez * ez;
            return (r2f < (same ? rcs2 : rcx2)) & (((accept >> ot) & 1u) != 0u) & ((o.tag >> 2) == rep);
        }
    };
    const std::false_type general{};
    // a candidate that passed the test (or, with `check`, one to test):
    // into the list unless it is chain-local.  The lanes of a wave that
    // append in the same call take their slots with one atomic between them.
    auto hit = [&](int q, bool check) {
        const BeadRec o = srec[q];
        bool keep = !check || test(o, general);
        // open edges: the fixed-point difference is exact only modulo 2^32
        // units, so a record of a far cell that shares a bucket with a
        // neighbour cell is rejected by its cell coordinates
        if (keep && any_open && open_any) {
            const int4 oc = scell[q];
            if ((!px && abs(oc.x - c[0]) > 1) || (!py && abs(oc.y - c[1]) > 1) || (!pz && abs(oc.z - c[2]) > 1))
                keep = false;
        }
        const int64_t j = keep ? (int64_t)sid[q] : i;
        keep = keep && !local_pair(ri, i, j);
        const uint64_t wave = __ballot(keep);
        if (!keep) return;
        const int leader = __builtin_ctzll(wave);
        const uint32_t lane = threadIdx.x & 63u;
        uint32_t base = 0u;
        if (lane == (uint32_t)leader) base = atomicAdd(&ctl->list_n, (uint32_t)__popcll(wave));
        base = (uint32_t)__shfl((int)base, leader, 64);
        const uint32_t slot = base + (uint32_t)__popcll(wave & ((1ull << lane) - 1ull));
        if (slot < cap) {
            PairRec pr;
            pr.i = (int32_t)i;
            pr.j = (int32_t)j;
            pr.rep = (int32_t)rep;
            pr.same = (((o.tag ^ mt) & 1u) == 0u) ? 1 : 0;
            a.b.plist[slot] = pr;
        }
    };

    const int total = s_tot[src];
    const uint32_t pk = s_pk[src];
    const uint32_t wrapped = s_wr[src];
    // the range of stream entry k < 127 is found by counting the bytes of the
    // packed s_pre[1..4] that are <= k (no borrow between bytes while k, pre
    // < 128); larger k take the plain search
    const int nfast = min(total, 127);
    // sorted position of stream entry k < nfast
    auto locate = [&](int k) -> int {
        uint32_t kb = (uint32_t)k | 0x80u;
        kb |= kb << 8;
        kb |= kb << 16;
        const int q = __popc((kb - pk) & 0x80808080u);
        return k + s_sh[q][src];
    };
    // The stream is screened without branches, SW entries at a time: the
    // entry index k is the same in every lane (so its byte pattern is scalar
    // arithmetic), a lane past the end of its own stream fetches some valid
    // record and ignores it, and a candidate within the list cutoff sets bit
    // k of the hit masks (k < 128); the hits are processed afterwards.
    const uint32_t last = (uint32_t)(a.n_nt - 1);
    uint64_t hit0 = 0, hit1 = 0;
    constexpr int SW = 4;  // entries per pass (a power of 2, so no pass straddles bit 64)
    auto screen = [&](auto fast) {
        for (int k0 = 0; k0 < nfast; k0 += SW) {
            BeadRec o[SW];
#pragma unroll
            for (int v = 0; v < SW; ++v) {
                const uint32_t at = (uint32_t)locate(k0 + v);
                o[v] = srec[min(at, last)];
            }
            uint32_t bits = 0u;
#pragma unroll
            for (int v = 0; v < SW; ++v) bits |= (uint32_t)test(o[v], fast) << v;
            if (k0 < 64) hit0 |= (uint64_t)bits << k0;
            else hit1 |= (uint64_t)bits << (k0 - 64);
        }
    };
    if (a.g.fast_screen) screen(std::true_type{});
    else screen(general);
    // entries past the lane's own stream
    if (nfast < 64) {
        hit0 &= (1ull << nfast) - 1ull;
        hit1 = 0;
    } else {
        hit1 &= (1ull << (nfast - 64)) - 1ull;
    }
    for (uint64_t h = hit0; h; h &= h - 1) hit(locate(__builtin_ctzll(h)), false);
    for (uint64_t h = hit1; h; h &= h - 1) hit(locate(64 + __builtin_ctzll(h)), false);
    for (int k = nfast; k < total; ++k) {
        int q = 0;
        for (int r = 1; r < 5; ++r) q = (k >= s_pre[r][src]) ? r : q;
        hit(k + s_sh[q][src], true);
    }
    // cells outside the fast stream: the neighbour across a periodic x face
    // (bit 8 + q), or every cell of a range that wraps the bucket array
    // (bit q, rare); their records are screened four per pass
    if (wrapped & 0x1F1Fu) {
        const int ncx = ri.ncell[0], ncy = ri.ncell[1], ncz = ri.ncell[2];
        auto wrap = [&](int v, int n, bool per_) { return per_ ? (v < 0 ? v + n : (v >= n ? v - n : v)) : v; };
        auto walk = [&](int lo, int hi) {
            for (int q0 = lo; q0 < hi; q0 += 4) {
                BeadRec o[4];
#pragma unroll
                for (int v = 0; v < 4; ++v) o[v] = srec[min(q0 + v, hi - 1)];
                uint32_t bits = 0u;
#pragma unroll
                for (int v = 0; v < 4; ++v) bits |= (uint32_t)((q0 + v < hi) & test(o[v], general)) << v;
                for (uint32_t b = bits; b; b &= b - 1) hit(q0 + __builtin_ctz(b), false);
            }
        };
        auto cell = [&](int cx, int cy, int cz) {
            const uint32_t kb = bucket_of(a.g, wrap(cx, ncx, px), cy, cz, (int)rep);
            walk(start[kb], start[kb + 1]);
        };
        const int dxlo = (wrapped & 0x20u) ? -1 : 0, dxhi = (wrapped & 0x40u) ? 1 : 0;
#pragma unroll 1
        for (int q = 0; q < 5; ++q) {
            const int dy = q == 0 ? 0 : (q == 1 ? 1 : q - 3), dz = q <= 1 ? 0 : 1;
            const int cy = wrap(c[1] + dy, ncy, py), cz = wrap(c[2] + dz, ncz, pz);
            if ((wrapped >> (8 + q)) & 1u) cell(c[0] == 0 ? -1 : c[0] + 1, cy, cz);
            if (!((wrapped >> q) & 1u)) continue;
            if (q == 0) {
                walk(p + 1, start[B.kown + 1]);
                cell(c[0] + 1, c[1], c[2]);
                continue;
            }
            for (int dx = dxlo; dx <= dxhi; ++dx) cell(c[0] + dx, cy, cz);
        }
    }
    }  // p < n_nt
    }  // record blocks
    // a list past its buffer stops the run at these positions; the host
    // enlarges it, rebuilds and continues
    __syncthreads();
    if (t == 0 && __hip_atomic_load(&ctl->list_n, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) > cap)
        atomicMax((unsigned long long *)&ctl->halt_step, (unsigned long long)built_step);
}

// ------------------------------------------------------------------- scan

__device__ __forceinline__ int wave_incl_scan(int v)
{
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        const int o = __shfl_up(v, d, 64);
        if ((threadIdx.x & 63) >= d) v += o;
    }
    return v;
}

// Exclusive scan of the 256 per-thread values of a workgroup; returns the
// thread's exclusive prefix and writes the workgroup total.
__device__ __forceinline__ int block_excl_scan(int v, int *total)
{
    __shared__ int wsum[4];
    const int incl = wave_incl_scan(v);
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    if (lane == 63) wsum[wv] = incl;
    __syncthreads();
    int base = 0;
    for (int k = 0; k < wv; ++k) base += wsum[k];
    *total = wsum[0] + wsum[1] + wsum[2] + wsum[3];
    __syncthreads();
    return base + incl - v;
}

// Total of each chunk of SCAN_CHUNK histogram entries.
__global__ void __launch_bounds__(256) k_scan_reduce(const uint32_t *__restrict__ count, int *__restrict__ bsum,
                                                     const Ctl *ctl)
{
    if (halted(*ctl, ctl->done_step + 1)) return;
    // 16 buckets (8 words) per thread
    const uint4 *c4 = reinterpret_cast<const uint4 *>(count + (int64_t)blockIdx.x * (SCAN_CHUNK / 2)) + threadIdx.x * 2;
    int v = 0;
#pragma unroll
    for (int k = 0; k < 2; ++k) {
        const uint4 q = c4[k];
        v += (int)((q.x & 0xFFFFu) + (q.x >> 16) + (q.y & 0xFFFFu) + (q.y >> 16) + (q.z & 0xFFFFu) + (q.z >> 16) +
                   (q.w & 0xFFFFu) + (q.w >> 16));
    }
    int total;
    block_excl_scan(v, &total);
    if (threadIdx.x == 0) bsum[blockIdx.x] = total;
}

// Offsets of one chunk of SCAN_CHUNK keys from the preceding chunk totals.
__global__ void __launch_bounds__(256) k_scan_down(const uint32_t *__restrict__ count, const int *__restrict__ bsum,
                                                   int *__restrict__ start, int nkeys, const Ctl *ctl)
{
    if (halted(*ctl, ctl->done_step + 1)) return;
    // the chunk's counts first (in flight while the offset is summed): 16
    // buckets in 8 words per thread
    const int64_t base = (int64_t)blockIdx.x * SCAN_CHUNK + threadIdx.x * 16;
    const uint4 *c4 = reinterpret_cast<const uint4 *>(count + base / 2);
    int v[16];
#pragma unroll
    for (int k = 0; k < 2; ++k) {
        const uint4 q = c4[k];
        const uint32_t w[4] = {q.x, q.y, q.z, q.w};
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            v[8 * k + 2 * j] = (int)(w[j] & 0xFFFFu);
            v[8 * k + 2 * j + 1] = (int)(w[j] >> 16);
        }
    }
    // offset of this chunk: sum of the preceding chunks' totals
    int pre = 0;
    const int nb = (int)blockIdx.x;
    for (int k0 = threadIdx.x; k0 < nb; k0 += 8 * (int)blockDim.x) {
        int w[8];  // eight loads in flight per pass
#pragma unroll
        for (int r = 0; r < 8; ++r) {
            const int k = k0 + r * (int)blockDim.x;
            w[r] = k < nb ? bsum[k] : 0;
        }
#pragma unroll
        for (int r = 0; r < 8; ++r) pre += w[r];
    }
    int ptot;
    block_excl_scan(pre, &ptot);
    int sum = 0;
#pragma unroll
    for (int k = 0; k < 16; ++k) sum += v[k];
    int tot;
    int run = ptot + block_excl_scan(sum, &tot);
    int4 *s4 = reinterpret_cast<int4 *>(start + base);
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        int4 o;
        o.x = run; run += v[4 * k];
        o.y = run; run += v[4 * k + 1];
        o.z = run; run += v[4 * k + 2];
        o.w = run; run += v[4 * k + 3];
        s4[k] = o;
    }
    if (blockIdx.x == gridDim.x - 1 && threadIdx.x == blockDim.x - 1) start[nkeys] = run;
}

// Counting-sort scatter: bead records into key order (grid-stride); empties
// the neighbour list for the build that follows.
__global__ void __launch_bounds__(256) k_scatter(const int *__restrict__ key, const int *__restrict__ slot,
                                                 const int *__restrict__ start, const BeadRec *__restrict__ rec,
                                                 const int4 *__restrict__ rcell, BeadRec *__restrict__ srec,
                                                 int *__restrict__ sid, int4 *__restrict__ scell, Ctl *ctl,
                                                 int64_t n, int any_open)
{
    if (halted(*ctl, ctl->done_step + 1)) return;
    if (blockIdx.x == 0 && threadIdx.x == 0) ctl->list_n = 0u;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const int k = key[i];
        const int p = start[k] + slot[i];
        srec[p] = rec[i];
        sid[p] = (int)i;
        if (any_open) scell[p] = rcell[i];
    }
}

// --------------------------------------------------------------- thermalize

__global__ void __launch_bounds__(WG_THREADS) k_thermalize(const StepArgs *__restrict__ A, double kT, uint64_t seed)
{
    const StepArgs &a = *A;
    const int tix = tile_index(a.n_tiles, a.n_tiles_pad);
    if (tix >= a.n_tiles) return;
    const Tile tile = cload(&a.b.tiles[tix]);
    const RepInfo &ri = a.b.rep[tile.rep];
    const int s = threadIdx.x & 1, n = threadIdx.x < TILE_NT ? tile.n0 + (int)(threadIdx.x >> 1) : tile.n_bp;
    if (n >= tile.n_bp) return;
    const int64_t i = ri.off + 2 * (int64_t)n + s;
    const int cur = a.b.ctl->par;
    const int64_t N = a.n_nt;
    double xi[6];
    noise6(seed, 0, 0, (uint32_t)i, 1u, xi);
    D3 V = v3(xi[0], xi[1], xi[2]) * sqrt(kT / a.ph.M);
    D3 L = v3(xi[3], xi[4], xi[5]) * sqrt(a.ph.I * kT);
    const D3 u = ld3(a.b.u[cur], N, i);
    L = L - u * dot(L, u);
    if ((ri.flags & REP_TETHER) && n == 0) {
        V = v3(0.0, 0.0, 0.0);
        L = V;
    }
    st3(a.b.V[cur], N, i, V);
    st3(a.b.L[cur], N, i, L);
    st3(a.b.Vf, N, i, V);
    st3(a.b.Lf, N, i, L);
}

// ------------------------------------------------ linking number, writhe

// The curves of each replica from the positions in buffer `buf`: strand 0
// beads, strand 1 beads and the centreline through the midpoints of the
// paired patches (Sec. 3.1), as FP64 points [n][3] per curve.  An open
// duplex's strands also get their closure points (appendix on the closure
// procedure), each from the thread of its end base pair: the end bead moved
// by `reach` along the unit tangent from the neighbouring bead of its strand
// outwards.  One workgroup per block of LK_THREADS base pairs of one set.
__global__ void __launch_bounds__(LK_THREADS) k_curves(const StepArgs *__restrict__ A, const CurveSet *__restrict__ sets,
                                                      const int2 *__restrict__ blocks, int n_pts, int buf,
                                                      double *__restrict__ curves)
{
    const StepArgs &a = *A;
    const int2 blk = blocks[blockIdx.x];
    const CurveSet cs = sets[blk.x];
    const int n = blk.y + (int)threadIdx.x;
    if (n >= cs.n_bp) return;
    auto beads = [&](int bp, D3 &q0, D3 &q1) {
        const int64_t j0 = cs.off + 2 * (int64_t)bp, j1 = j0 + 1;
        q0 = bead_of(ld3(a.b.R[buf], a.n_nt, j0), ld3(a.b.u[buf], a.n_nt, j0), a.ph.db);
        q1 = bead_of(ld3(a.b.R[buf], a.n_nt, j1), ld3(a.b.u[buf], a.n_nt, j1), a.ph.db);
    };
    const int64_t i0 = cs.off + 2 * (int64_t)n, i1 = i0 + 1;
    const D3 R0 = ld3(a.b.R[buf], a.n_nt, i0), u0 = ld3(a.b.u[buf], a.n_nt, i0);
    const D3 R1 = ld3(a.b.R[buf], a.n_nt, i1), u1 = ld3(a.b.u[buf], a.n_nt, i1);
    const D3 b0 = bead_of(R0, u0, a.ph.db), b1 = bead_of(R1, u1, a.ph.db);
    const D3 c = (patch_of(R0, u0, a.ph.dp) + patch_of(R1, u1, a.ph.dp)) * 0.5;
    double *pA = curves + 3 * ((int64_t)cs.pt0 + n);
    double *pB = pA + 3 * (int64_t)n_pts, *pC = pB + 3 * (int64_t)n_pts;
    pA[0] = b0.x; pA[1] = b0.y; pA[2] = b0.z;
    pB[0] = b1.x; pB[1] = b1.y; pB[2] = b1.z;
    pC[0] = c.x; pC[1] = c.y; pC[2] = c.z;
    if (cs.open && cs.n_bp >= 2 && (n == 0 || n == cs.n_bp - 1)) {
        D3 q0, q1;
        beads(n == 0 ? 1 : n - 1, q0, q1);
        const D3 d0 = b0 - q0, d1 = b1 - q1;
        const D3 e0 = b0 + d0 * (cs.reach / sqrt(dot(d0, d0))), e1 = b1 + d1 * (cs.reach / sqrt(dot(d1, d1)));
        // slot n_bp: after the last bead; slot n_bp + 1: before the first
        const int64_t slot = n == 0 ? cs.n_bp + 1 : cs.n_bp;
        double *qA = curves + 3 * ((int64_t)cs.pt0 + slot), *qB = qA + 3 * (int64_t)n_pts;
        qA[0] = e0.x; qA[1] = e0.y; qA[2] = e0.z;
        qB[0] = e1.x; qB[1] = e1.y; qB[2] = e1.z;
    }
}

// Half the signed solid angle of the spherical triangle with vertices along
// x, y, z (lengths lx, ly, lz) as the point (den, num) whose argument it is:
// tan(Omega/2) = x.(y x z) / (lx ly lz + (x.y) lz + (x.z) ly + (y.z) lx)
// (Van Oosterom and Strackee, IEEE Trans. Biomed. Eng. 30, 125 (1983)).
__device__ __forceinline__ void tri_half(D3 x, D3 y, D3 z, double lx, double ly, double lz, double &num, double &den)
{
    num = dot(x, cross(y, z));
    den = lx * ly * lz + dot(x, y) * lz + dot(x, z) * ly + dot(y, z) * lx;
}

// Gauss's double integral (appendix on the closure procedure) over segment
// p1 -> p2 of one closed polygon and segment p3 -> p4 of another, times
// 4 pi.  The integrand is the pull-back of the area form of the sphere by
// (r_1 - r_2)/|r_1 - r_2| up to sign, so the pair integral is the signed
// area of the geodesic quadrangle with corners p1-p3, p2-p3, p2-p4, p1-p4;
// written with r_ij = p_j - p_i it is the fan of two triangles below.  The
// difference vectors of two disjoint segments fill a parallelogram that
// misses the origin, so they lie in an open half-space and the area is below
// 2 pi: the two half-angles add as the argument of the product of their
// points, one atan2 for the pair.
__device__ __forceinline__ double pair_omega(D3 p1, D3 p2, D3 p3, D3 p4)
{
    const D3 r13 = p3 - p1, r14 = p4 - p1, r23 = p3 - p2, r24 = p4 - p2;
    const double l13 = sqrt(dot(r13, r13)), l14 = sqrt(dot(r14, r14));
    const double l23 = sqrt(dot(r23, r23)), l24 = sqrt(dot(r24, r24));
    double y1, x1, y2, x2;
    tri_half(r13, r23, r24, l13, l23, l24, y1, x1);
    tri_half(r13, r24, r14, l13, l24, l14, y2, x2);
    return 2.0 * atan2(y1 * x2 + y2 * x1, x1 * x2 - y1 * y2);
}

// Row sums of the segment-pair solid angles of one curve set, for the rows
// i0 .. i0 + LK_THREADS - 1.  Thread i holds segment i -> i+1 (mod nS) of the
// closed strand curve A (nS points) and segment i -> i+1 of the centreline C
// (nC points, closed unless c_open); curve B (nS points, closed) and C
// stream through LDS in chunks of LK_THREADS segments.  Sums over the rows
// of Omega(A_i, B_j) over all j (the linking number) and of Omega(C_i, C_j)
// over the j whose segment shares no vertex with segment i, each unordered
// pair once: on a closed C the half window j - i = 2 .. nC/2 (mod nC), the
// antipodal j - i = nC/2 of an even curve only from i < nC/2; on an open C
// the segments j >= i + 2 (the writhe), reduced in a fixed order to part[2].
// Called by all threads of a workgroup.
__device__ void gauss_rows(const double *__restrict__ cA, const double *__restrict__ cB,
                           const double *__restrict__ cC, int nS, int nC, int c_open, int i0,
                           double *__restrict__ part)
{
    __shared__ double sB[LK_THREADS + 1][3];
    __shared__ double sC[LK_THREADS + 1][3];
    __shared__ double red[LK_THREADS][2];
    const int t = threadIdx.x;
    const int i = i0 + t;
    const int segC = c_open ? nC - 1 : nC;  // centreline segments
    const bool rowA = i < nS, rowC = i < segC;
    D3 a0 = v3(0.0, 0.0, 0.0), a1 = a0, c0 = a0, c1 = a0;
    if (rowA) {
        const int i1 = i + 1 == nS ? 0 : i + 1;
        a0 = v3(cA[3 * i], cA[3 * i + 1], cA[3 * i + 2]);
        a1 = v3(cA[3 * i1], cA[3 * i1 + 1], cA[3 * i1 + 2]);
    }
    if (rowC) {
        const int i1 = i + 1 == nC ? 0 : i + 1;
        c0 = v3(cC[3 * i], cC[3 * i + 1], cC[3 * i + 2]);
        c1 = v3(cC[3 * i1], cC[3 * i1 + 1], cC[3 * i1 + 2]);
    }
    double lk = 0.0, wr = 0.0;
    const int rows = nS > segC ? nS : segC;
    for (int j0 = 0; j0 < rows; j0 += LK_THREADS) {
        const int mB = max(0, min(LK_THREADS, nS - j0));    // segments of B in this chunk
        const int mC = max(0, min(LK_THREADS, segC - j0));  // segments of C in this chunk
        __syncthreads();
        for (int q = t; q <= max(mB, mC); q += LK_THREADS) {  // m + 1 points, the last may wrap
            if (mB > 0 && q <= mB) {
                const int j = j0 + q == nS ? 0 : j0 + q;
                sB[q][0] = cB[3 * j]; sB[q][1] = cB[3 * j + 1]; sB[q][2] = cB[3 * j + 2];
            }
            if (mC > 0 && q <= mC) {
                const int j = j0 + q == nC ? 0 : j0 + q;
                sC[q][0] = cC[3 * j]; sC[q][1] = cC[3 * j + 1]; sC[q][2] = cC[3 * j + 2];
            }
        }
        __syncthreads();
        if (rowA)
            for (int q = 0; q < mB; ++q) lk += pair_omega(a0, a1, lds3(sB, q), lds3(sB, q + 1));
        if (rowC)
            for (int q = 0; q < mC; ++q) {
                const int j = j0 + q;
                bool take;
                if (c_open) {
                    take = j >= i + 2;
                } else {
                    const int d = j >= i ? j - i : j - i + nC;  // (j - i) mod nC
                    take = d >= 2 && d <= nC - 2 && (2 * d < nC || (2 * d == nC && 2 * i < nC));
                }
                if (take) wr += pair_omega(c0, c1, lds3(sC, q), lds3(sC, q + 1));
            }
    }
    red[t][0] = lk;
    red[t][1] = wr;
    for (int w = LK_THREADS / 2; w > 0; w >>= 1) {
        __syncthreads();
        if (t < w) {
            red[t][0] += red[t + w][0];
            red[t][1] += red[t + w][1];
        }
    }
    if (t == 0) {
        part[0] = red[0][0];
        part[1] = red[0][1];
    }
}

// Rings of a context: one workgroup per block of LK_THREADS base pairs of
// one ring (the curves of k_curves), partial[block][2].
__global__ void __launch_bounds__(LK_THREADS) k_gauss(const CurveSet *__restrict__ sets, const int2 *__restrict__ blocks,
                                                     int n_pts, const double *__restrict__ curves,
                                                     double *__restrict__ partial)
{
    const int2 blk = blocks[blockIdx.x];
    const CurveSet cs = sets[blk.x];
    const double *cA = curves + 3 * (int64_t)cs.pt0;
    const double *cB = cA + 3 * (int64_t)n_pts, *cC = cB + 3 * (int64_t)n_pts;
    gauss_rows(cA, cB, cC, cs.n_str, cs.n_bp, cs.open, blk.y, partial + 2 * blockIdx.x);
}

// Per ring, in block order: Lk = (sum of its rows) / (4 pi) and Wr twice the
// sum of its rows over 4 pi (the rows hold each unordered pair once, the
// integral over the torus counts it twice).
__device__ __forceinline__ void gauss_total(const double *__restrict__ partial, int blk0, int n_blk,
                                            double *__restrict__ out)
{
    double lk = 0.0, wr = 0.0;
    for (int b = 0; b < n_blk; ++b) {
        lk += partial[2 * (blk0 + b)];
        wr += partial[2 * (blk0 + b) + 1];
    }
    const double k = 0.25 / 3.14159265358979323846;
    out[0] = lk * k;
    out[1] = 2.0 * wr * k;
}

__global__ void __launch_bounds__(64) k_gauss_sum(const CurveSet *__restrict__ sets, int n_sets,
                                                 const double *__restrict__ partial, double *__restrict__ out)
{
    const int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= n_sets) return;
    const CurveSet cs = sets[r];
    gauss_total(partial, cs.blk0, cs.n_blk, out + 2 * r);
}

// One ring given as three closed curves of n points each (A, B: the two
// strands; C: the centreline): workgroup b takes the rows from b LK_THREADS
// on; then the fixed-order total.
__global__ void __launch_bounds__(LK_THREADS) k_gauss_curves(const double *__restrict__ A, const double *__restrict__ B,
                                                            const double *__restrict__ C, int n,
                                                            double *__restrict__ partial)
{
    gauss_rows(A, B, C, n, n, 0, (int)blockIdx.x * LK_THREADS, partial + 2 * blockIdx.x);
}

__global__ void __launch_bounds__(64) k_gauss_curves_sum(const double *__restrict__ partial, int n_blk,
                                                        double *__restrict__ out)
{
    if (blockIdx.x == 0 && threadIdx.x == 0) gauss_total(partial, 0, n_blk, out);
}

// --------------------------------------------------------------- diagnostics

// Per-term forces and energies of the positions in buffer `which`, plus the
// kinetic energies of the velocities Vk, Lk (the full-step ones): per tile,
// energies in a fixed-order reduction into eacc[tile][DSDNA_NENERGY].
template <typename real, bool DAMP>
__global__ void __launch_bounds__(WG_THREADS) k_diag(const StepArgs *__restrict__ A, int which, uint32_t mask,
                                                    const double *__restrict__ Vk, const double *__restrict__ Lk)
{
    __shared__ TileLds<real> S;
    __shared__ double red[DSDNA_NENERGY][WG_THREADS / 64];
    const StepArgs &a = *A;
    // the cell list is only valid when the binning before this launch
    // completed without error
    if (a.b.ctl->code != 0) return;
    const int tix = tile_index(a.n_tiles, a.n_tiles_pad);
    if (tix >= a.n_tiles) return;
    const Tile tile = cload(&a.b.tiles[tix]);
    const RepInfo &ri = a.b.rep[tile.rep];
    double e[DSDNA_NENERGY];
    for (int k = 0; k < DSDNA_NENERGY; ++k) e[k] = 0.0;
    const int64_t step = a.b.ctl->step;
    const StagedSite site = load_site(a, ri, tile, which);
    const int s = threadIdx.x & 1, bl = threadIdx.x >> 1, n = threadIdx.x < TILE_NT ? tile.n0 + bl : tile.n_bp;
    const bool flagged = contact_flag(a, tix);
    const V3<real> fexv = (n < tile.n_bp && flagged) ? take_fex<real>(a, site.i) : v3<real>(0, 0, 0);
    stage_site(a, S, site);
    SiteForces<real> f = tile_forces<real, DAMP>(a, S, ri, tile, fexv, mask, step, e);
    if (n < tile.n_bp) {
        const int64_t i = ri.off + 2 * (int64_t)n + s;
        a.b.diag_fb[3 * i] = (double)f.b.x;
        a.b.diag_fb[3 * i + 1] = (double)f.b.y;
        a.b.diag_fb[3 * i + 2] = (double)f.b.z;
        a.b.diag_fp[3 * i] = (double)f.p.x;
        a.b.diag_fp[3 * i + 1] = (double)f.p.y;
        a.b.diag_fp[3 * i + 2] = (double)f.p.z;
        if (s == 0) a.b.open[ri.off / 2 + n] = S.sOpen[bl + HALO_BP];
        // kinetic energies of the rigid body: M V^2 / 2 and L^2 / (2 I)
        const D3 V = ld3(Vk, a.n_nt, i), L = ld3(Lk, a.n_nt, i);
        e[DSDNA_NTERMS] = 0.5 * a.ph.M * dot(V, V);
        e[DSDNA_NTERMS + 1] = 0.5 * dot(L, L) * a.ph.inv_I;
    }
    // per-tile energy partials: fixed-order reduction
    for (int k = 0; k < DSDNA_NENERGY; ++k) {
        double v = e[k];
        for (int d = 32; d >= 1; d >>= 1) v += __shfl_xor(v, d, 64);
        if ((threadIdx.x & 63) == 0) red[k][threadIdx.x >> 6] = v;
    }
    __syncthreads();
    if (threadIdx.x < DSDNA_NENERGY) {
        double v = 0.0;
        for (int w = 0; w < WG_THREADS / 64; ++w) v += red[threadIdx.x][w];
        a.b.eacc[(int64_t)tix * DSDNA_NENERGY + threadIdx.x] = v;
    }
}

// Tiles of replica r: the first and the number of them.
__device__ __forceinline__ int2 replica_tiles(const RepInfo &ri) { return make_int2(ri.tile0, (ri.n_bp + TILE_BP - 1) / TILE_BP); }

// Per replica, the energy partials of its tiles summed in a fixed order
// (thread t takes tiles t, t + 256, ...; then a fixed tree):
// out[r][DSDNA_NENERGY].  One workgroup per replica.
__global__ void __launch_bounds__(256) k_rep_energy(const StepArgs *__restrict__ A, double *__restrict__ out)
{
    __shared__ double red[256];
    const StepArgs &a = *A;
    const int r = blockIdx.x, t = threadIdx.x;
    const int2 tl = replica_tiles(a.b.rep[r]);
    for (int k = 0; k < DSDNA_NENERGY; ++k) {
        double v = 0.0;
        for (int q = t; q < tl.y; q += 256) v += a.b.eacc[(int64_t)(tl.x + q) * DSDNA_NENERGY + k];
        red[t] = v;
        for (int w = 128; w > 0; w >>= 1) {
            __syncthreads();
            if (t < w) red[t] += red[t + w];
        }
        __syncthreads();
        if (t == 0) out[(int64_t)r * DSDNA_NENERGY + k] = red[0];
        __syncthreads();
    }
}

// Bubbles (Sec. 5: maximal runs of open base pairs), per tile of the open
// flags: hist[tile][nhist] counts the runs inside the tile that touch
// neither of its ends (length k, k >= nhist - 1 in the last bin); info[tile]
// = (open run at its start, open run at its end, open base pairs, base
// pairs).  One thread per tile.
__global__ void __launch_bounds__(64) k_bubble_tiles(const StepArgs *__restrict__ A, int nhist,
                                                    int32_t *__restrict__ hist, int4 *__restrict__ info)
{
    const StepArgs &a = *A;
    const int tix = blockIdx.x * blockDim.x + threadIdx.x;
    if (tix >= a.n_tiles) return;
    const Tile tile = cload(&a.b.tiles[tix]);
    const RepInfo &ri = a.b.rep[tile.rep];
    const int len = min(TILE_BP, tile.n_bp - tile.n0);
    const uint8_t *op = a.b.open + ri.off / 2 + tile.n0;
    int32_t *h = hist + (int64_t)tix * nhist;
    for (int k = 0; k < nhist; ++k) h[k] = 0;
    int lead = 0;
    while (lead < len && op[lead]) ++lead;
    int nopen = lead, q = lead, trail = 0;
    if (lead == len) {
        trail = len;
    } else {
        while (q < len) {
            if (!op[q]) {
                ++q;
                continue;
            }
            int e = q;
            while (e < len && op[e]) ++e;
            nopen += e - q;
            if (e == len) trail = e - q;  // touches the end: counted across tiles
            else h[min(e - q, nhist - 1)] += 1;
            q = e;
        }
    }
    info[tix] = make_int4(lead, trail, nopen, len);
}

// Per replica: the interior runs of its tiles summed bin by bin in tile
// order, then the runs across tile boundaries by one thread walking the
// tiles (an open run continues through all-open tiles; on a ring the run at
// the end joins the run at the start, and an all-open ring is one run):
// frac[r] = open fraction, out[r][nhist].  One workgroup per replica.
__global__ void __launch_bounds__(256) k_bubble_rep(const StepArgs *__restrict__ A, int nhist,
                                                   const int32_t *__restrict__ hist, const int4 *__restrict__ info,
                                                   double *__restrict__ frac, int64_t *__restrict__ out)
{
    extern __shared__ int64_t sh[];  // nhist bins
    const StepArgs &a = *A;
    const int r = blockIdx.x, t = threadIdx.x;
    const RepInfo &ri = a.b.rep[r];
    const int2 tl = replica_tiles(ri);
    for (int k = t; k < nhist; k += blockDim.x) {
        int64_t v = 0;
        for (int q = 0; q < tl.y; ++q) v += hist[(int64_t)(tl.x + q) * nhist + k];
        sh[k] = v;
    }
    __syncthreads();
    if (t == 0) {
        const auto bin = [nhist](int64_t len) { return (int)(len < nhist - 1 ? len : nhist - 1); };
        const bool ring = ri.flags & REP_RING;
        int64_t nopen = 0, carry = 0, first = -1;  // first: the open run at the replica's start
        bool all_open = true;
        for (int q = 0; q < tl.y; ++q) {
            const int4 in = info[tl.x + q];
            nopen += in.z;
            if (in.x == in.w) {  // an all-open tile: the run goes on
                carry += in.w;
                continue;
            }
            all_open = false;
            const int64_t run = carry + in.x;  // the run that ends at this tile's first closed bp
            if (first < 0) first = run;
            else if (run > 0) sh[bin(run)] += 1;
            carry = in.y;
        }
        if (all_open) {
            if (ri.n_bp > 0) sh[bin(ri.n_bp)] += 1;
        } else if (ring) {
            if (carry + first > 0) sh[bin(carry + first)] += 1;
        } else {
            if (first > 0) sh[bin(first)] += 1;
            if (carry > 0) sh[bin(carry)] += 1;
        }
        frac[r] = ri.n_bp > 0 ? (double)nopen / (double)ri.n_bp : 0.0;
    }
    __syncthreads();
    for (int k = t; k < nhist; k += blockDim.x) out[(int64_t)r * nhist + k] = sh[k];
}

// ---------------------------------------------------------------- launchers

static dim3 tiles_grid(const StepArgs &a) { return dim3((unsigned)a.n_tiles_pad); }

// Workgroups of `kernel` (with `threads` threads) resident on the current
// device at once, rounded down to a multiple of 8 (at least 8); cached per
// device and kernel.
static int resident_workgroups(const void *kernel, int threads)
{
    static std::mutex mu;
    static std::map<std::pair<int, const void *>, int> known;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 8;
    std::lock_guard<std::mutex> lock(mu);
    const auto key = std::make_pair(dev, kernel);
    const auto it = known.find(key);
    if (it != known.end()) return it->second;
    int per_cu = 0, cus = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, threads, 0) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
        return 8;
    const int g = std::max(8, per_cu * cus / 8 * 8);
    known[key] = g;
    return g;
}

// Grid of a rebuild kernel over `items` work items: at most REBUILD_GRID
// workgroups, a multiple of 8 (the XCD-aware grid-stride loops need it).
static dim3 rebuild_grid(int64_t items)
{
    const int64_t g = std::min<int64_t>(std::max<int64_t>(items, 1), REBUILD_GRID);
    return dim3((unsigned)((g + 7) / 8 * 8));
}

hipError_t launch_bin(const StepArgs &a, const StepArgs *dA, int which, hipStream_t s)
{
    hipLaunchKernelGGL(k_bin, rebuild_grid(a.n_tiles_pad), dim3(WG_THREADS), 0, s, dA, which);
    return hipGetLastError();
}

hipError_t launch_scan(const StepArgs &a, hipStream_t s)
{
    const int nkeys = a.g.nbucket;
    const int nchunk = nkeys / SCAN_CHUNK;
    hipLaunchKernelGGL(k_scan_reduce, dim3(nchunk), dim3(256), 0, s, a.b.count, a.b.bsum, a.b.ctl);
    hipLaunchKernelGGL(k_scan_down, dim3(nchunk), dim3(256), 0, s, a.b.count, a.b.bsum, a.b.start, nkeys, a.b.ctl);
    return hipGetLastError();
}

hipError_t launch_scatter(const StepArgs &a, hipStream_t s)
{
    hipLaunchKernelGGL(k_scatter, rebuild_grid((a.n_nt + 255) / 256), dim3(256), 0, s, a.b.key, a.b.slot, a.b.start,
                       a.b.rec, a.b.rcell, a.b.srec, a.b.sid, a.b.scell, a.b.ctl, a.n_nt, a.g.any_open);
    return hipGetLastError();
}

// The list build runs as many workgroups as are resident at once, each
// walking its share of the record blocks: its per-workgroup set-up (control
// block, arguments, the histogram clear) is paid once per workgroup, and no
// workgroup waits for a slot behind the first wave of them.
hipError_t launch_build(const StepArgs &a, const StepArgs *dA, hipStream_t s)
{
    const int64_t nblk = (a.n_nt + EXCL_THREADS - 1) / EXCL_THREADS;
    const void *k = a.g.any_open ? reinterpret_cast<const void *>(k_build<true>)
                                 : reinterpret_cast<const void *>(k_build<false>);
    const dim3 g((unsigned)std::min<int64_t>((nblk + 7) / 8 * 8, resident_workgroups(k, EXCL_THREADS)));
    if (a.g.any_open)
        hipLaunchKernelGGL(k_build<true>, g, dim3(EXCL_THREADS), 0, s, dA, a.b.srec, a.b.sid, a.b.scell, a.b.start);
    else
        hipLaunchKernelGGL(k_build<false>, g, dim3(EXCL_THREADS), 0, s, dA, a.b.srec, a.b.sid, a.b.scell, a.b.start);
    return hipGetLastError();
}

// Threads of the pair kernel: the list holds a few pairs per thousand beads.
constexpr int PAIRS_GRID = 256;

hipError_t launch_pairs(const StepArgs &a, const StepArgs *dA, int which, int energy, int mode, hipStream_t s)
{
    (void)a;
    hipLaunchKernelGGL(k_pairs, dim3(PAIRS_GRID), dim3(256), 0, s, dA, which, energy, mode);
    return hipGetLastError();
}

hipError_t launch_step(const StepArgs &a, const StepArgs *dA, int fp64, int mode, int write_full, int rebuild_after,
                       int age, hipStream_t s)
{
    const bool damp = a.ph.dihedral_damping != 0;
#define DSDNA_LAUNCH_STEP(R, D)                                                                             \
    hipLaunchKernelGGL((k_step<R, D>), tiles_grid(a), dim3(WG_THREADS), 0, s, dA, mode, write_full, rebuild_after, \
                       age)
    if (fp64 && damp) DSDNA_LAUNCH_STEP(double, true);
    else if (fp64) DSDNA_LAUNCH_STEP(double, false);
    else if (damp) DSDNA_LAUNCH_STEP(float, true);
    else DSDNA_LAUNCH_STEP(float, false);
#undef DSDNA_LAUNCH_STEP
    return hipGetLastError();
}

hipError_t launch_thermalize(const StepArgs &a, const StepArgs *dA, double kT, uint64_t seed, hipStream_t s)
{
    hipLaunchKernelGGL(k_thermalize, tiles_grid(a), dim3(WG_THREADS), 0, s, dA, kT, seed);
    return hipGetLastError();
}

hipError_t launch_diag(const StepArgs &a, const StepArgs *dA, int which, int fp64, uint32_t term_mask,
                       const double *Vk, const double *Lk, hipStream_t s)
{
    const bool damp = a.ph.dihedral_damping != 0;
#define DSDNA_LAUNCH_DIAG(R, D) \
    hipLaunchKernelGGL((k_diag<R, D>), tiles_grid(a), dim3(WG_THREADS), 0, s, dA, which, term_mask, Vk, Lk)
    if (fp64 && damp) DSDNA_LAUNCH_DIAG(double, true);
    else if (fp64) DSDNA_LAUNCH_DIAG(double, false);
    else if (damp) DSDNA_LAUNCH_DIAG(float, true);
    else DSDNA_LAUNCH_DIAG(float, false);
#undef DSDNA_LAUNCH_DIAG
    return hipGetLastError();
}

hipError_t launch_rep_energy(const StepArgs &a, const StepArgs *dA, double *out, int n_rep, hipStream_t s)
{
    (void)a;
    hipLaunchKernelGGL(k_rep_energy, dim3(n_rep), dim3(256), 0, s, dA, out);
    return hipGetLastError();
}

hipError_t launch_bubbles(const StepArgs &a, const StepArgs *dA, int nhist, int32_t *hist_tiles, int4 *info,
                          double *frac, int64_t *out, int n_rep, hipStream_t s)
{
    hipLaunchKernelGGL(k_bubble_tiles, dim3((a.n_tiles + 63) / 64), dim3(64), 0, s, dA, nhist, hist_tiles, info);
    hipLaunchKernelGGL(k_bubble_rep, dim3(n_rep), dim3(256), sizeof(int64_t) * (size_t)nhist, s, dA, nhist,
                       hist_tiles, info, frac, out);
    return hipGetLastError();
}

hipError_t launch_linking_curves(const double *A, const double *B, const double *C, int n, double *partial,
                                 double *out, hipStream_t s)
{
    const int n_blk = (n + LK_THREADS - 1) / LK_THREADS;
    hipLaunchKernelGGL(k_gauss_curves, dim3(n_blk), dim3(LK_THREADS), 0, s, A, B, C, n, partial);
    hipLaunchKernelGGL(k_gauss_curves_sum, dim3(1), dim3(64), 0, s, partial, n_blk, out);
    return hipGetLastError();
}

hipError_t launch_linking(const StepArgs *dA, int which, const CurveSet *sets, int n_sets, const int2 *blocks,
                          int n_blocks, int n_pts, double *curves, double *partial, double *out, hipStream_t s,
                          hipEvent_t ev0, hipEvent_t ev1)
{
    if (n_blocks <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_curves, dim3(n_blocks), dim3(LK_THREADS), 0, s, dA, sets, blocks, n_pts, which, curves);
    if (ev0) (void)hipEventRecord(ev0, s);
    hipLaunchKernelGGL(k_gauss, dim3(n_blocks), dim3(LK_THREADS), 0, s, sets, blocks, n_pts, curves, partial);
    if (ev1) (void)hipEventRecord(ev1, s);
    hipLaunchKernelGGL(k_gauss_sum, dim3((n_sets + 63) / 64), dim3(64), 0, s, sets, n_sets, partial, out);
    return hipGetLastError();
}

}  // namespace dsdna
