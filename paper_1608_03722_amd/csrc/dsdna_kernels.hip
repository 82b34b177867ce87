// dsdna_kernels.hip -- gfx950 kernels of one Langevin time step of the
// single-nucleotide dsDNA model (Fosado et al., arXiv:1608.03722).
//
// Per step (all kernels read the step index and the buffer parity from the
// device control block, so a captured graph replays unchanged):
//   k_step     one workgroup per tile of TILE_BP base pairs of one replica:
//              stage the tile's FP64 sites in LDS, evaluate every
//              fixed-topology term once into LDS outboxes, gather them per
//              site (no atomics), add each bead's excluded volume from the
//              cell list (fixed-point accumulation, order independent), the
//              external loads and the Langevin forces, then integrate the
//              rigid body (FP64) and bin its new bead position (histogram
//              atomics: the counting-sort count phase).
//   k_scan_*   exclusive scan of the histogram (counting-sort offsets)
//   k_scatter  counting-sort scatter of the bead records into key order;
//              clears the histogram for the next step.
#include <hip/hip_runtime.h>
#include <math.h>
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

__device__ __forceinline__ D3 ld3(const double *soa, int64_t n, int64_t i)
{
    return v3(soa[i], soa[n + i], soa[2 * n + i]);
}
__device__ __forceinline__ void st3(double *soa, int64_t n, int64_t i, D3 a)
{
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
        const uint32_t lo0 = 0xD2511F53u * c.x, hi0 = __umulhi(0xD2511F53u, c.x);
        const uint32_t lo1 = 0xCD9E8D57u * c.z, hi1 = __umulhi(0xCD9E8D57u, c.z);
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
// so the radius keeps its relative accuracy near u = 1.
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
        const uint32_t a = w[k];
        const float lnu = a < 0x80000000u ? logf(((float)a + 0.5f) * 0x1p-32f)
                                          : log1pf(-(((float)(0xFFFFFFFFu - a) + 0.5f) * 0x1p-32f));
        const float rad = sqrtf(-2.0f * lnu);
        const float ang = 6.28318530717958648f * (((float)w[k + 1] + 0.5f) * 0x1p-32f);
        float s, c;
        sincosf(ang, &s, &c);
        xi[k] = rad * c;
        xi[k + 1] = rad * s;
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

// --------------------------------------------------------------- cell list

// Cell of a bead and its 16-bit neighbour coordinates.  Periodic dims:
// wrapped into [0, L), cell = floor(frac * ncell), coordinate = frac * 2^16;
// open dims: relative to the replica origin, cell = floor(x / h), coordinate
// = x * 256 modulo 2^16.  Returns false if the position is not finite or too
// far from the origin to be binned.
__device__ __forceinline__ bool cell_of(const RepInfo &ri, D3 p, int c[3], uint32_t qc[3])
{
    const double x[3] = {p.x - ri.lo[0], p.y - ri.lo[1], p.z - ri.lo[2]};
    bool ok = true;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        if (ri.flags & (REP_PER_X << k)) {
            double t = x[k] * ri.inv_len[k];
            ok = ok && isfinite(t);
            t = ok ? t - floor(t) : 0.0;
            int ci = (int)(t * (double)ri.ncell[k]);
            ci = ci >= ri.ncell[k] ? ri.ncell[k] - 1 : (ci < 0 ? 0 : ci);
            c[k] = ci;
            qc[k] = (uint32_t)(t * 65536.0) & 0xFFFFu;
        } else {
            ok = ok && (fabs(x[k]) < 1.0e6);  // also rejects NaN
            const double xs = ok ? x[k] : 0.0;
            c[k] = (int)floor(xs * ri.inv_h[k]);
            qc[k] = (uint32_t)(long long)rint(xs * OPEN_Q_INV) & 0xFFFFu;
        }
    }
    return ok;
}

__device__ __forceinline__ uint32_t bucket_of(const Grid &g, int cx, int cy, int cz, int rep)
{
    return ((uint32_t)cx + g.A * (uint32_t)cy + g.B * (uint32_t)cz + g.C * (uint32_t)rep) & g.mask;
}

// 16-bit tag: strand (bit 0), steric (bit 1), replica modulo 2^14 (bits 2..15).
__device__ __forceinline__ uint32_t make_tag(int rep, int n, int s)
{
    return (((uint32_t)rep & 0x3FFFu) << 2) | ((n % 3 == 0) ? 2u : 0u) | (uint32_t)s;
}

// Bin one bead: record, counting-sort key (bucket in its strand's plane) and
// slot within the key (histogram).
__device__ __forceinline__ void insert_bead(const StepArgs &a, const RepInfo &ri, int rep, int n, int s,
                                            int64_t i, D3 bead, int64_t step)
{
    int c[3];
    uint32_t qc[3];
    if (!cell_of(ri, bead, c, qc)) {
        raise_error(a.b.ctl, isfinite(bead.x + bead.y + bead.z) ? DSDNA_EDOMAIN : DSDNA_ENAN, step, i);
        c[0] = c[1] = c[2] = 0;
    }
    const uint32_t key = bucket_of(a.g, c[0], c[1], c[2], rep) + (uint32_t)s * (uint32_t)a.g.nbucket;
    a.b.rec[i] = make_uint2(qc[0] | (qc[1] << 16), qc[2] | (make_tag(rep, n, s) << 16));
    a.b.key[i] = (int32_t)key;
    a.b.slot[i] = atomicAdd(&a.b.count[key], 1);
}

// ------------------------------------------------------------- tile stage

template <typename real>
struct TileLds {
    double sB[TILE_NT + 4 * HALO_BP][3];   // FP64 sites, halo of 2 bp each side
    double sP[TILE_NT + 4 * HALO_BP][3];
    real oStep[2][TILE_BP + 1][4][3];      // per strand, per backbone step m
    real oBend[2][TILE_BP + 2][3][3];      // per strand, per bending centre
    real oHb[TILE_BP][3];                  // force on strand-0 patch
    uint8_t sOpen[TILE_BP + 2 * HALO_BP];  // open flags of bp n0-2 .. n0+129
    real sW[TILE_NT][3];                   // excluded-volume force per nucleotide
    uint8_t perm[TILE_NT];                 // search order: steric beads first
    int wcnt[2][TILE_NT / 64];             // per-wave steric / ghost counts
};

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

typedef short short2v __attribute__((ext_vector_type(2)));

// All conservative and external site forces of the calling thread's
// nucleotide, restricted to the terms in `mask`.  Must be called by all
// threads of the workgroup (it synchronises).  With energies != nullptr the
// per-term energies owned by this thread are added there (diagnostics only).
template <typename real>
__device__ __forceinline__ SiteForces<real> tile_forces(const StepArgs &a, TileLds<real> &S, const RepInfo &ri, int rep, int n0,
                                        int cur, uint32_t mask, int64_t step, double *energies)
{
    const int t = threadIdx.x;
    const int64_t N = a.n_nt;
    const Phys &ph = a.ph;
    const int nbp = ri.n_bp;
    const double *Rc = a.b.R[cur];
    const double *uc = a.b.u[cur];

    // --- stage FP64 sites of the tile and its halo (LDS index l <-> bp
    //     n0 - 2 + l/2, strand l & 1)
    for (int l = t; l < TILE_NT + 4 * HALO_BP; l += blockDim.x) {
        const int bp = n0 - HALO_BP + (l >> 1);
        if (bp >= 0 && bp < nbp) {
            const int64_t i = ri.off + 2 * (int64_t)bp + (l & 1);
            const D3 R = ld3(Rc, N, i), u = ld3(uc, N, i);
            const D3 b = bead_of(R, u, ph.db), p = patch_of(R, u, ph.dp);
            S.sB[l][0] = b.x; S.sB[l][1] = b.y; S.sB[l][2] = b.z;
            S.sP[l][0] = p.x; S.sP[l][1] = p.y; S.sP[l][2] = p.z;
        }
    }
    __syncthreads();

    // --- hydrogen bonds and open flags (truncated harmonic between the
    //     patches of a base pair, Appendix A)
    const double k2s = ri.k2_scale;
    for (int q = t; q < TILE_BP + 2 * HALO_BP; q += blockDim.x) {
        const int bp = n0 - HALO_BP + q;
        uint8_t open = 0;
        V3<real> f = v3<real>(0, 0, 0);
        if (bp >= 0 && bp < nbp) {
            const D3 d64 = lds3(S.sP, 2 * q + 1) - lds3(S.sP, 2 * q);
            const double r = sqrt(dot(d64, d64));
            open = r > ph.rc_hb;
            if (!open && (mask & (1u << DSDNA_TERM_HBOND))) {
                const real pref = (real)(ph.hb_pref * k2s);
                const real c = (ph.r0_hb == 0.0) ? (real)2 * pref : (real)2 * pref * ((real)1 - (real)(ph.r0_hb / r));
                f = cvt<real>(d64) * c;
                if (energies && q >= HALO_BP && q < TILE_BP + HALO_BP)
                    energies[DSDNA_TERM_HBOND] += ph.hb_pref * k2s *
                        ((r - ph.r0_hb) * (r - ph.r0_hb) - (ph.rc_hb - ph.r0_hb) * (ph.rc_hb - ph.r0_hb));
            }
        }
        S.sOpen[q] = open;
        if (q >= HALO_BP && q < TILE_BP + HALO_BP) put3(S.oHb[q - HALO_BP], f);
    }
    __syncthreads();

    const bool rule = ph.ssdna_rule != 0;
    // --- backbone steps: FENE + WCA core, Morse, dihedral, planarity on the
    //     pair of nucleotides (s, m), (s, m+1), m = n0 - 1 + mi
    for (int q = t; q < 2 * (TILE_BP + 1); q += blockDim.x) {
        const int s = q & 1, mi = q >> 1, m = n0 - 1 + mi;
        V3<real> fBa = v3<real>(0, 0, 0), fPa = fBa, fBb = fBa, fPb = fBa;
        if (m >= 0 && m + 1 < nbp) {
            const int la = 2 * (mi + 1) + s, lb = la + 2;
            const D3 Ba = lds3(S.sB, la), Pa = lds3(S.sP, la), Bb = lds3(S.sB, lb), Pb = lds3(S.sP, lb);
            const bool own = mi >= 1;  // step m belongs to the tile that holds nucleotide m
            // backbone: FENE + WCA(eps_bb, sig_bb) between consecutive beads
            if (mask & (1u << DSDNA_TERM_BOND)) {
                const D3 d64 = Bb - Ba;
                const double r2 = dot(d64, d64);
                if (r2 >= ph.R0 * ph.R0) {
                    raise_error(a.b.ctl, DSDNA_EBOND, step, ri.off + 2 * (int64_t)m + s);
                } else {
                    // FENE attraction and the WCA core cancel to a few percent
                    // near the bond minimum, so (dU/dr)/r is formed in FP64
                    const double x = 1.0 - r2 / (ph.R0 * ph.R0);
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
                const D3 d64 = Pb - Pa;
                const V3<real> d = cvt<real>(d64);
                const real ir = rsq(dot(d, d));
                const real r = dot(d, d) * ir;
                const real ex = exp(-(real)ph.lam * (r - (real)ph.r0_m));
                const V3<real> f = d * ((real)(2.0 * ph.K4 * ph.lam) * ex * ((real)1 - ex) * ir);
                fPa = fPa + f;
                fPb = fPb - f;
                if (energies && own) {
                    const double r64 = sqrt(dot(d64, d64)), e64 = exp(-ph.lam * (r64 - ph.r0_m));
                    energies[DSDNA_TERM_STACK] += ph.K4 * (1.0 - e64) * (1.0 - e64);
                }
            }
            const V3<real> b1 = cvt<real>(Pa - Ba), b2 = cvt<real>(Pb - Pa), b3 = cvt<real>(Bb - Pb);
            // helical twist: dihedral of (B_m, P_m, P_m+1, B_m+1); gradient as in
            // Blondel & Karplus (1996), free of the 1/sin(phi) singularity
            const bool masked = rule && S.sOpen[mi + 1] && S.sOpen[mi + 2] && (S.sOpen[mi] || S.sOpen[mi + 3]);
            if ((mask & (1u << DSDNA_TERM_TWIST)) && !masked) {
                const V3<real> A = cross(b1, b2), B = cross(b2, b3);
                const real AA = dot(A, A), BB = dot(B, B), GG = dot(b2, b2);
                const real iG = rsq(GG), lG = GG * iG;
                const real inv = rsq(AA * BB);
                const real cphi = dot(A, B) * inv, sphi = lG * dot(b1, B) * inv;
                const real cd = (real)ph.cos_d, sd = (real)ph.sin_d;
                // -dU/dphi = K3 sin(phi - d)
                const real mdU = (real)ph.K3 * (sphi * cd - cphi * sd);
                const real FG = dot(b1, b2), HG = -dot(b3, b2);
                const real iAA = rcp(AA), iBB = rcp(BB);
                const V3<real> tA = A * (lG * iAA), tB = B * (lG * iBB);
                const V3<real> sA = A * (FG * iAA * iG), sB = B * (HG * iBB * iG);
                fBa = fBa + (-tA) * mdU;
                fPa = fPa + (tA + sA - sB) * mdU;
                fPb = fPb + (-tB - sA + sB) * mdU;
                fBb = fBb + tB * mdU;
                if (energies && own) energies[DSDNA_TERM_TWIST] += ph.K3 * (1.0 + (double)cphi * ph.cos_d + (double)sphi * ph.sin_d);
            }
            // planarity: angle at P_m+1 between P_m and B_m+1, (K5/2)(alpha - a0)^2
            if (mask & (1u << DSDNA_TERM_PLANAR)) {
                const V3<real> r1 = -b2, r2 = b3;
                const real l11 = dot(r1, r1), l22 = dot(r2, r2);
                const real il = rsq(l11 * l22);
                real c = dot(r1, r2) * il;
                c = c > (real)1 ? (real)1 : (c < (real)-1 ? (real)-1 : c);
                const real al = acos(c);
                const real sn = sqrt((real)1 - c * c);
                const real dUdc = -(real)ph.K5 * (al - (real)ph.a0) * rcp(sn);
                const V3<real> dca = r2 * il - r1 * (c * rcp(l11)), dcc = r1 * il - r2 * (c * rcp(l22));
                const V3<real> fa = dca * (-dUdc), fc = dcc * (-dUdc);
                fPa = fPa + fa;
                fBb = fBb + fc;
                fPb = fPb - (fa + fc);
                if (energies && own) energies[DSDNA_TERM_PLANAR] += 0.5 * ph.K5 * ((double)al - ph.a0) * ((double)al - ph.a0);
            }
        }
        put3(S.oStep[s][mi][0], fBa);
        put3(S.oStep[s][mi][1], fPa);
        put3(S.oStep[s][mi][2], fBb);
        put3(S.oStep[s][mi][3], fPb);
    }
    // --- Kratky-Porod bending on patches (s, m-1), (s, m), (s, m+1)
    for (int q = t; q < 2 * (TILE_BP + 2); q += blockDim.x) {
        const int s = q & 1, mi = q >> 1, m = n0 - 1 + mi;
        V3<real> f0 = v3<real>(0, 0, 0), f1 = f0, f2 = f0;
        const bool masked = rule && S.sOpen[mi] && S.sOpen[mi + 1] && S.sOpen[mi + 2];
        if ((mask & (1u << DSDNA_TERM_BEND)) && m >= 1 && m + 1 < nbp && !masked) {
            const int la = 2 * mi + s;
            const D3 Pa = lds3(S.sP, la), Pc = lds3(S.sP, la + 2), Pe = lds3(S.sP, la + 4);
            const V3<real> r1 = cvt<real>(Pa - Pc), r2 = cvt<real>(Pe - Pc);
            const real l11 = dot(r1, r1), l22 = dot(r2, r2);
            const real il = rsq(l11 * l22);
            const real c = dot(r1, r2) * il;
            const real K6 = (real)ph.K6;
            f0 = (r2 * il - r1 * (c * rcp(l11))) * (-K6);
            f2 = (r1 * il - r2 * (c * rcp(l22))) * (-K6);
            f1 = -(f0 + f2);
            if (energies && mi >= 1 && mi <= TILE_BP) energies[DSDNA_TERM_BEND] += ph.K6 * (1.0 + (double)c);
        }
        put3(S.oBend[s][mi][0], f0);
        put3(S.oBend[s][mi][1], f1);
        put3(S.oBend[s][mi][2], f2);
    }
    __syncthreads();

    // --- gather per site (fixed order, no atomics)
    const int s = t & 1, bl = t >> 1, n = n0 + bl;
    const int nbp_tile = min(TILE_BP, nbp - n0);
    SiteForces<real> out;
    out.b = v3<real>(0, 0, 0);
    out.p = out.b;
    if (n < nbp) {
        out.b = get3(S.oStep[s][bl][2]) + get3(S.oStep[s][bl + 1][0]);
        out.p = get3(S.oStep[s][bl][3]) + get3(S.oStep[s][bl + 1][1]) + get3(S.oBend[s][bl][2]) +
                get3(S.oBend[s][bl + 1][1]) + get3(S.oBend[s][bl + 2][0]);
        const V3<real> hb = get3(S.oHb[bl]);
        out.p = s == 0 ? out.p + hb : out.p - hb;
    }

    // --- excluded volume (WCA, steric/ghost rule of Sec. 2).  Every bead
    //     scans the other strand's bucket plane (cross-strand pairs, any bead
    //     type); steric beads also scan their own strand's plane (steric
    //     pairs).  Searched in an order that puts the steric beads in the
    //     first waves; forces go back to the natural order through LDS.
    if (mask & (1u << DSDNA_TERM_EXCL)) {
        {
            const bool valid = bl < nbp_tile;
            const bool st = valid && ((n % 3) == 0);
            const uint64_t bs = __ballot(st), bg = __ballot(valid && !st);
            const int lane = t & 63, w = t >> 6;
            const uint64_t below = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
            if (lane == 0) {
                S.wcnt[0][w] = __popcll(bs);
                S.wcnt[1][w] = __popcll(bg);
            }
            __syncthreads();
            int os = 0, og = 0, nst = 0;
            for (int k = 0; k < TILE_NT / 64; ++k) {
                if (k < w) { os += S.wcnt[0][k]; og += S.wcnt[1][k]; }
                nst += S.wcnt[0][k];
            }
            if (st) S.perm[os + __popcll(bs & below)] = (uint8_t)t;
            else if (valid) S.perm[nst + og + __popcll(bg & below)] = (uint8_t)t;
        }
        __syncthreads();
        if (t < 2 * nbp_tile) {
            const int lw = S.perm[t];
            const int sw = lw & 1, nw = n0 + (lw >> 1);
            const int64_t iw = ri.off + 2 * (int64_t)nw + sw;
            const D3 bw = lds3(S.sB, lw + 2 * HALO_BP);
            int c[3];
            uint32_t mq[3];
            cell_of(ri, bw, c, mq);
            const bool mysteric = (nw % 3) == 0;
            const uint32_t myrep = (uint32_t)rep & 0x3FFFu;
            const float rs = (float)ph.rc_s + a.g.margin, rx = (float)ph.rc_x + a.g.margin;
            const float rs2 = rs * rs, rx2 = rx * rx;
            const real rcs2 = (real)(ph.rc_s * ph.rc_s), rcx2 = (real)(ph.rc_x * ph.rc_x);
            const real sig_s2 = (real)(ph.sig_s * ph.sig_s), sig_x2 = (real)(ph.sig_x * ph.sig_x);
            const bool px = ri.flags & REP_PER_X, py = ri.flags & REP_PER_Y, pz = ri.flags & REP_PER_Z;
            const float qx = ri.q[0], qy = ri.q[1], qz = ri.q[2];
            const bool qint = ri.qsame != 0;
            const int64_t jlo = ri.off, jhi = ri.off + 2 * (int64_t)nbp;
            const short2v mxy = __builtin_bit_cast(short2v, mq[0] | (mq[1] << 16));
            long long ax = 0, ay = 0, az = 0;  // fixed point, 2^-32 units: order independent
            double e_excl = 0.0;
            const double *Rcj = a.b.R[cur], *ucj = a.b.u[cur];
            const uint2 *__restrict__ srec = a.b.srec;

            // exact test and force for a candidate that passed the 16-bit
            // pre-check (rare: true contacts and the slack shell)
            auto refine = [&](int p, bool same) {
                const int j = a.b.sid[p];
                if (j == (int)iw || j < jlo || j >= jhi) return;   // itself, other replica
                const D3 bj = bead_of(ld3(Rcj, N, j), ld3(ucj, N, j), ph.db);
                D3 d64 = bj - bw;
                if (px) d64.x -= ri.len[0] * rint(d64.x * ri.inv_len[0]);
                if (py) d64.y -= ri.len[1] * rint(d64.y * ri.inv_len[1]);
                if (pz) d64.z -= ri.len[2] * rint(d64.z * ri.inv_len[2]);
                const V3<real> d = cvt<real>(d64);
                const real r2 = dot(d, d);
                if (r2 >= (same ? rcs2 : rcx2)) return;
                const real ir2 = rcp(r2);
                const real sr2 = (same ? sig_s2 : sig_x2) * ir2;
                const real sr6 = sr2 * sr2 * sr2;
                const real g = (real)(24.0 * ph.eps) * ((real)2 * sr6 * sr6 - sr6) * ir2;
                const double fx = (double)(g * d.x), fy = (double)(g * d.y), fz = (double)(g * d.z);
                if (!(fabs(fx) + fabs(fy) + fabs(fz) < 1.0e9)) {  // overlapping beads: out of range
                    raise_error(a.b.ctl, DSDNA_ENAN, step, iw);
                    return;
                }
                // force on the bead = -g d (repulsive)
                ax -= __double2ll_rn(fx * 4294967296.0);
                ay -= __double2ll_rn(fy * 4294967296.0);
                az -= __double2ll_rn(fz * 4294967296.0);
                if (energies) {
                    const double s2 = (same ? ph.sig_s * ph.sig_s : ph.sig_x * ph.sig_x) / dot(d64, d64);
                    const double s6 = s2 * s2 * s2;
                    e_excl += 0.5 * 4.0 * ph.eps * (s6 * s6 - s6 + 0.25);
                }
            };
            // 16-bit pre-check of one record: replica and type, then the
            // squared distance in coordinate units (integer when the unit is
            // the same along x, y and z)
            auto precheck = [&](const uint2 o, bool same, int t2) -> bool {
                const uint32_t tj = o.y >> 16;
                if ((tj >> 2) != myrep) return false;
                if (same && !(tj & 2u)) return false;
                if (qint) {
                    const short2v dxy = __builtin_bit_cast(short2v, o.x) - mxy;
                    const int dz = (int)(short)(uint16_t)(o.y - mq[2]);
                    return __builtin_amdgcn_sdot2(dxy, dxy, dz * dz, false) < t2;
                }
                const float dx = (float)(int16_t)(uint16_t)((o.x & 0xFFFFu) - mq[0]) * qx;
                const float dy = (float)(int16_t)(uint16_t)((o.x >> 16) - mq[1]) * qy;
                const float dz = (float)(int16_t)(uint16_t)((o.y & 0xFFFFu) - mq[2]) * qz;
                return dx * dx + dy * dy + dz * dz < (same ? rs2 : rx2);
            };

            // nine rows of three cells (dz, dy; cx-1..cx+1): three consecutive
            // buckets each unless the row wraps (periodic x or bucket index)
            const int ncx = ri.ncell[0], ncy = ri.ncell[1], ncz = ri.ncell[2];
            const bool xwrap = px && (c[0] == 0 || c[0] == ncx - 1);
            uint32_t kr[9];
#pragma unroll
            for (int q = 0; q < 9; ++q) {
                int cy = c[1] + (q % 3) - 1, cz = c[2] + (q / 3) - 1;
                if (py) cy = cy < 0 ? cy + ncy : (cy >= ncy ? cy - ncy : cy);
                if (pz) cz = cz < 0 ? cz + ncz : (cz >= ncz ? cz - ncz : cz);
                kr[q] = bucket_of(a.g, c[0] - 1, cy, cz, rep);
            }
            // pass 0: the other strand's plane (every bead); pass 1: the own
            // strand's plane (steric beads only)
            for (int pass = 0; pass < (mysteric ? 2 : 1); ++pass) {
                const bool same = pass == 1;
                const int t2 = same ? ri.t2_same : ri.t2_cross;
                const uint32_t plane = (uint32_t)(same ? sw : 1 - sw) * (uint32_t)a.g.nbucket;
                // stream position k of range q sits at k + sh[q] in the sorted
                // records; pre[q] = first stream position of range q
                int sh[9], pre[9];
                int total = 0;
#pragma unroll
                for (int q = 0; q < 9; ++q) {
                    const bool reg = !xwrap && kr[q] + 2u <= a.g.mask;
                    const int l0 = reg ? a.b.start[plane + kr[q]] : 0;
                    const int h0 = reg ? a.b.start[plane + kr[q] + 3] : 0;
                    pre[q] = total;
                    sh[q] = l0 - total;
                    total += h0 - l0;
                }
                // the nine ranges as one candidate stream, four independent
                // loads per trip (the wave runs max over lanes of the total)
                constexpr int U = 4;
                for (int k0 = 0; k0 < total; k0 += U) {
                    uint2 o[U];
                    int pp[U];
#pragma unroll
                    for (int v = 0; v < U; ++v) {
                        const int k = k0 + v < total ? k0 + v : total - 1;
                        int d = sh[0];
#pragma unroll
                        for (int r = 1; r < 9; ++r) d = (k >= pre[r]) ? sh[r] : d;
                        pp[v] = k + d;
                        o[v] = srec[pp[v]];
                    }
#pragma unroll
                    for (int v = 0; v < U; ++v)
                        if (k0 + v < total && precheck(o[v], same, t2)) refine(pp[v], same);
                }
                // rows that wrap: cell by cell (rare)
                for (int q = 0; q < 9; ++q) {
                    int cy = c[1] + (q % 3) - 1, cz = c[2] + (q / 3) - 1;
                    if (py) cy = cy < 0 ? cy + ncy : (cy >= ncy ? cy - ncy : cy);
                    if (pz) cz = cz < 0 ? cz + ncz : (cz >= ncz ? cz - ncz : cz);
                    if (!xwrap && bucket_of(a.g, c[0] - 1, cy, cz, rep) + 2u <= a.g.mask) continue;
                    for (int dx = -1; dx <= 1; ++dx) {
                        int cx = c[0] + dx;
                        if (px) cx = cx < 0 ? cx + ncx : (cx >= ncx ? cx - ncx : cx);
                        const uint32_t kb = plane + bucket_of(a.g, cx, cy, cz, rep);
                        for (int p = a.b.start[kb]; p < a.b.start[kb + 1]; ++p)
                            if (precheck(srec[p], same, t2)) refine(p, same);
                    }
                }
            }
            put3(S.sW[lw], v3<real>((real)((double)ax * 0x1p-32), (real)((double)ay * 0x1p-32),
                                    (real)((double)az * 0x1p-32)));
            if (energies) energies[DSDNA_TERM_EXCL] += e_excl;
        }
        __syncthreads();
        if (n < nbp) out.b = out.b + get3(S.sW[t]);
    }
    if (n >= nbp) return out;

    const int l = t + 2 * HALO_BP;
    const D3 bi = lds3(S.sB, l);
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
                const D3 b0 = lds3(S.sB, l - s), b1 = lds3(S.sB, l - s + 1);
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

// ------------------------------------------------------------------- tiles

__device__ __forceinline__ int tile_index(int n_tiles, int n_tiles_pad)
{
    // consecutive workgroups go to the 8 XCDs in turn; give each XCD a
    // contiguous run of tiles so chain neighbours share an L2
    const int per = n_tiles_pad >> 3;
    const int b = blockIdx.x;
    return (b & 7) * per + (b >> 3);
}

// Rotation of the axis of a free linear rotor by th about unit k:
// u cos th + (k x u) sin th + k (k.u)(1 - cos th).  cos and sin come from
// their Taylor series through th^10 for th < 1/32 (error below 1e-19),
// otherwise from sincos.
__device__ __forceinline__ D3 rotate(D3 u, D3 k, double th)
{
    double sn, cs;
    if (th < 0.03125) {
        const double t2 = th * th;
        cs = 1.0 - t2 * (1.0 / 2 - t2 * (1.0 / 24 - t2 * (1.0 / 720 - t2 * (1.0 / 40320 - t2 * (1.0 / 3628800)))));
        sn = th * (1.0 - t2 * (1.0 / 6 - t2 * (1.0 / 120 - t2 * (1.0 / 5040 - t2 * (1.0 / 362880)))));
    } else {
        sincos(th, &sn, &cs);
    }
    return u * cs + cross(k, u) * sn + k * (dot(k, u) * (1.0 - cs));
}

// ---------------------------------------------------------------- k_step

template <typename real>
__global__ void __launch_bounds__(TILE_NT, 4) k_step(const StepArgs *__restrict__ A, int mode, int write_full)
{
    __shared__ TileLds<real> S;
    const StepArgs &a = *A;
    const Ctl ctl = *a.b.ctl;
    if (ctl.code != 0) return;
    const int tix = tile_index(a.n_tiles, a.n_tiles_pad);
    if (tix >= a.n_tiles) return;
    const Tile tile = a.b.tiles[tix];
    const RepInfo &ri = a.b.rep[tile.rep];
    const int cur = ctl.par, nxt = cur ^ 1;
    const int64_t step = ctl.step;
    const int64_t N = a.n_nt;
    const Phys &ph = a.ph;

    SiteForces<real> f;
    f.b = v3<real>(0, 0, 0);
    f.p = f.b;
    if (mode != MODE_FROM_FORCES) f = tile_forces<real>(a, S, ri, tile.rep, tile.n0, cur, ALL_TERMS, step, nullptr);

    const int s = threadIdx.x & 1, n = tile.n0 + (threadIdx.x >> 1);
    if (n >= ri.n_bp) return;
    const int64_t i = ri.off + 2 * (int64_t)n + s;
    D3 R = ld3(a.b.R[cur], N, i), u = ld3(a.b.u[cur], N, i);
    D3 V = ld3(a.b.V[cur], N, i), L = ld3(a.b.L[cur], N, i);
    const bool frozen = (ri.flags & REP_TETHER) && n == 0;

    D3 fb, fp;  // total site forces of this step
    if (mode == MODE_FROM_FORCES) {
        fb = ld3(a.b.Fb, N, i);
        fp = ld3(a.b.Fp, N, i);
    } else {
        V3<real> lb = v3<real>(0, 0, 0), lp = lb;
        if (!frozen && ph.gamma > 0.0) {
            // Langevin forces (Appendix A) per site: friction on the site's
            // velocity on the rigid body plus counter-based noise
            const D3 w = L * (1.0 / ph.I);
            const D3 vb = V + cross(w, u * (-ph.db)), vp = V + cross(w, u * ph.dp);
            if (sizeof(real) == sizeof(double)) {
                double xi[6];
                noise6(ph.seed, ph.noise_kind, (uint64_t)step, (uint32_t)i, 0u, xi);
                lb = cvt<real>(vb * (-ph.gamma) + v3(xi[0], xi[1], xi[2]) * ph.noise_amp);
                lp = cvt<real>(vp * (-ph.gamma) + v3(xi[3], xi[4], xi[5]) * ph.noise_amp);
            } else {
                float xi[6];
                noise6f(ph.seed, ph.noise_kind, (uint64_t)step, (uint32_t)i, 0u, xi);
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
        }
    } else {
        const D3 F = fb + fp;
        const D3 tau = cross(u, fp * ph.dp - fb * ph.db);
        const double km = ph.kick / ph.M;
        if (mode == MODE_NORMAL) {  // second half kick of the previous step
            V = V + F * km;
            L = L + tau * ph.kick;
        }
        if (write_full) {
            st3(a.b.Vf, N, i, V);
            st3(a.b.Lf, N, i, L);
            st3(a.b.Fb, N, i, fb);
            st3(a.b.Fp, N, i, fp);
        }
        // first half kick, drift, free rotation of the linear rotor
        V = V + F * km;
        L = L + tau * ph.kick;
        R = R + V * ph.dt;
        const D3 w = L * (1.0 / ph.I);
        const double wl = sqrt(dot(w, w));
        if (wl > 0.0) u = rotate(u, w * (1.0 / wl), wl * ph.dt);
        u = u * (1.0 / sqrt(dot(u, u)));
        L = L - u * dot(L, u);
    }
    st3(a.b.R[nxt], N, i, R);
    st3(a.b.u[nxt], N, i, u);
    st3(a.b.V[nxt], N, i, V);
    st3(a.b.L[nxt], N, i, L);
    if (!(isfinite(R.x + R.y + R.z) && isfinite(u.x + u.y + u.z))) raise_error(a.b.ctl, DSDNA_ENAN, step + 1, i);
    insert_bead(a, ri, tile.rep, n, s, i, bead_of(R, u, ph.db), step + 1);
}

// ------------------------------------------------------------ binning only

// Bins the beads of buffer `which` (after the state was set from the host).
__global__ void __launch_bounds__(256) k_bin(const StepArgs *__restrict__ A, int which)
{
    const StepArgs &a = *A;
    const int tix = tile_index(a.n_tiles, a.n_tiles_pad);
    if (tix >= a.n_tiles) return;
    const Tile tile = a.b.tiles[tix];
    const RepInfo &ri = a.b.rep[tile.rep];
    const int s = threadIdx.x & 1, n = tile.n0 + (threadIdx.x >> 1);
    if (n >= ri.n_bp) return;
    const int64_t i = ri.off + 2 * (int64_t)n + s;
    const D3 R = ld3(a.b.R[which], a.n_nt, i), u = ld3(a.b.u[which], a.n_nt, i);
    insert_bead(a, ri, tile.rep, n, s, i, bead_of(R, u, a.ph.db), a.b.ctl->step);
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

__global__ void __launch_bounds__(256) k_scan_reduce(const int *__restrict__ count, int *__restrict__ bsum,
                                                     const Ctl *ctl)
{
    if (ctl->code != 0) return;
    const int4 *c4 = reinterpret_cast<const int4 *>(count + (int64_t)blockIdx.x * SCAN_CHUNK) + threadIdx.x * 4;
    int v = 0;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const int4 q = c4[k];
        v += q.x + q.y + q.z + q.w;
    }
    int total;
    block_excl_scan(v, &total);
    if (threadIdx.x == 0) bsum[blockIdx.x] = total;
}

__global__ void __launch_bounds__(256) k_scan_down(const int *__restrict__ count, const int *__restrict__ bsum,
                                                   int *__restrict__ start, int nkeys, const Ctl *ctl)
{
    if (ctl->code != 0) return;
    // offset of this chunk: sum of the preceding chunks' totals
    int pre = 0;
    for (int k = threadIdx.x; k < (int)blockIdx.x; k += blockDim.x) pre += bsum[k];
    int ptot;
    block_excl_scan(pre, &ptot);
    const int64_t base = (int64_t)blockIdx.x * SCAN_CHUNK + threadIdx.x * 16;
    const int4 *c4 = reinterpret_cast<const int4 *>(count + base);
    int v[16];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const int4 q = c4[k];
        v[4 * k] = q.x; v[4 * k + 1] = q.y; v[4 * k + 2] = q.z; v[4 * k + 3] = q.w;
    }
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

// Counting-sort scatter: bead records (and their nucleotide ids) into key
// order; clears the histogram entries it used.  inc: also advance the step
// and flip the position buffers.
__global__ void __launch_bounds__(256) k_scatter(const int *__restrict__ key, const int *__restrict__ slot,
                                                 const int *__restrict__ start, const uint2 *__restrict__ rec,
                                                 uint2 *__restrict__ srec, int *__restrict__ sid,
                                                 int *__restrict__ count, Ctl *ctl, int64_t n, int inc)
{
    if (ctl->code != 0) return;
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) {
        const int k = key[i];
        const int p = start[k] + slot[i];
        srec[p] = rec[i];
        sid[p] = (int)i;
        count[k] = 0;
    }
    if (inc && i == 0) {
        ctl->step += 1;
        ctl->par ^= 1;
    }
}

// --------------------------------------------------------------- thermalize

__global__ void __launch_bounds__(256) k_thermalize(const StepArgs *__restrict__ A, double kT, uint64_t seed)
{
    const StepArgs &a = *A;
    const int tix = tile_index(a.n_tiles, a.n_tiles_pad);
    if (tix >= a.n_tiles) return;
    const Tile tile = a.b.tiles[tix];
    const RepInfo &ri = a.b.rep[tile.rep];
    const int s = threadIdx.x & 1, n = tile.n0 + (threadIdx.x >> 1);
    if (n >= ri.n_bp) return;
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

// --------------------------------------------------------------- diagnostics

template <typename real>
__global__ void __launch_bounds__(TILE_NT) k_diag(const StepArgs *__restrict__ A, int which, uint32_t mask)
{
    __shared__ TileLds<real> S;
    __shared__ double red[DSDNA_NTERMS][TILE_NT / 64];
    const StepArgs &a = *A;
    // the cell list is only valid when the binning before this launch
    // completed without error
    if (a.b.ctl->code != 0) return;
    const int tix = tile_index(a.n_tiles, a.n_tiles_pad);
    if (tix >= a.n_tiles) return;
    const Tile tile = a.b.tiles[tix];
    const RepInfo &ri = a.b.rep[tile.rep];
    double e[DSDNA_NTERMS];
    for (int k = 0; k < DSDNA_NTERMS; ++k) e[k] = 0.0;
    const int64_t step = a.b.ctl->step;
    SiteForces<real> f = tile_forces<real>(a, S, ri, tile.rep, tile.n0, which, mask, step, e);
    const int s = threadIdx.x & 1, bl = threadIdx.x >> 1, n = tile.n0 + bl;
    if (n < ri.n_bp) {
        const int64_t i = ri.off + 2 * (int64_t)n + s;
        a.b.diag_fb[3 * i] = (double)f.b.x;
        a.b.diag_fb[3 * i + 1] = (double)f.b.y;
        a.b.diag_fb[3 * i + 2] = (double)f.b.z;
        a.b.diag_fp[3 * i] = (double)f.p.x;
        a.b.diag_fp[3 * i + 1] = (double)f.p.y;
        a.b.diag_fp[3 * i + 2] = (double)f.p.z;
        if (s == 0) a.b.open[ri.off / 2 + n] = S.sOpen[bl + HALO_BP];
    }
    // per-tile energy partials: fixed-order reduction
    for (int k = 0; k < DSDNA_NTERMS; ++k) {
        double v = e[k];
        for (int d = 32; d >= 1; d >>= 1) v += __shfl_xor(v, d, 64);
        if ((threadIdx.x & 63) == 0) red[k][threadIdx.x >> 6] = v;
    }
    __syncthreads();
    if (threadIdx.x < DSDNA_NTERMS) {
        double v = 0.0;
        for (int w = 0; w < TILE_NT / 64; ++w) v += red[threadIdx.x][w];
        a.b.eacc[(int64_t)tix * DSDNA_NTERMS + threadIdx.x] = v;
    }
}

// ---------------------------------------------------------------- launchers

static dim3 tiles_grid(const StepArgs &a) { return dim3((unsigned)a.n_tiles_pad); }

hipError_t launch_bin(const StepArgs &a, const StepArgs *dA, int which, hipStream_t s)
{
    hipLaunchKernelGGL(k_bin, tiles_grid(a), dim3(TILE_NT), 0, s, dA, which);
    return hipGetLastError();
}

hipError_t launch_scan(const StepArgs &a, hipStream_t s)
{
    const int nkeys = 2 * a.g.nbucket;  // one plane of buckets per strand
    const int nchunk = nkeys / SCAN_CHUNK;
    hipLaunchKernelGGL(k_scan_reduce, dim3(nchunk), dim3(256), 0, s, a.b.count, a.b.bsum, a.b.ctl);
    hipLaunchKernelGGL(k_scan_down, dim3(nchunk), dim3(256), 0, s, a.b.count, a.b.bsum, a.b.start, nkeys,
                       a.b.ctl);
    return hipGetLastError();
}

hipError_t launch_scatter(const StepArgs &a, int inc_step, hipStream_t s)
{
    const unsigned nb = (unsigned)((a.n_nt + 255) / 256);
    hipLaunchKernelGGL(k_scatter, dim3(nb), dim3(256), 0, s, a.b.key, a.b.slot, a.b.start, a.b.rec, a.b.srec,
                       a.b.sid, a.b.count, a.b.ctl, a.n_nt, inc_step);
    return hipGetLastError();
}

hipError_t launch_step(const StepArgs &a, const StepArgs *dA, int fp64, int mode, int write_full, hipStream_t s)
{
    if (fp64)
        hipLaunchKernelGGL(k_step<double>, tiles_grid(a), dim3(TILE_NT), 0, s, dA, mode, write_full);
    else
        hipLaunchKernelGGL(k_step<float>, tiles_grid(a), dim3(TILE_NT), 0, s, dA, mode, write_full);
    return hipGetLastError();
}

hipError_t launch_thermalize(const StepArgs &a, const StepArgs *dA, double kT, uint64_t seed, hipStream_t s)
{
    hipLaunchKernelGGL(k_thermalize, tiles_grid(a), dim3(TILE_NT), 0, s, dA, kT, seed);
    return hipGetLastError();
}

hipError_t launch_diag(const StepArgs &a, const StepArgs *dA, int which, int fp64, uint32_t term_mask,
                       hipStream_t s)
{
    if (fp64)
        hipLaunchKernelGGL(k_diag<double>, tiles_grid(a), dim3(TILE_NT), 0, s, dA, which, term_mask);
    else
        hipLaunchKernelGGL(k_diag<float>, tiles_grid(a), dim3(TILE_NT), 0, s, dA, which, term_mask);
    return hipGetLastError();
}

}  // namespace dsdna
