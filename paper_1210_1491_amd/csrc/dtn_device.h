// Device primitives for the walk-on-spheres kernels (CDNA4, wave64).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "dtn_internal.h"

namespace dtn {

constexpr int kWave = 64;

// ------------------------------------------------------------------ Philox
// Philox4x32-10 (Salmon, Moraes, Dror & Shaw, SC'11): ten rounds of the
// two-multiplier S-box with the key bumped by the Weyl constants between
// rounds.  The 32x32->64 products map to v_mad_u64_u32; the key schedule is
// wave-uniform and stays in SGPRs.
struct Philox4 {
    uint32_t x, y, z, w;
};

// Three-input XOR in one VALU op: v_bitop3_b32 with truth table 0x96
// (a ^ b ^ c); the compiler does not form it from C xors here.
__device__ __forceinline__ uint32_t xor3(uint32_t a, uint32_t b, uint32_t c)
{
    return __builtin_amdgcn_bitop3_b32(a, b, c, 0x96);
}

__device__ __forceinline__ Philox4 philox4x32_10(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3,
                                                 uint32_t k0, uint32_t k1)
{
    // The keys are wave-uniform.  The empty statement makes them look new at
    // every call, so the ten round keys are recomputed by scalar adds here
    // instead of being kept live in 20 SGPRs across the walk loop (which
    // spills SGPRs into VGPR lanes and costs a v_readlane per use).
    asm volatile("" : "+s"(k0), "+s"(k1));
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        const uint64_t p0 = (uint64_t)0xD2511F53u * (uint64_t)c0;
        const uint64_t p1 = (uint64_t)0xCD9E8D57u * (uint64_t)c2;
        const uint32_t n0 = xor3((uint32_t)(p1 >> 32), c1, k0);
        // in the first round c3 (the stream id) and k1 are both wave-uniform:
        // their XOR is one scalar op and the vector side a two-input XOR
        // (a three-input one could read only one of them from a scalar register)
        const uint32_t n2 = r == 0 ? (uint32_t)(p0 >> 32) ^ (c3 ^ k1) : xor3((uint32_t)(p0 >> 32), c3, k1);
        c1 = (uint32_t)p1;
        c3 = (uint32_t)p0;
        c0 = n0;
        c2 = n2;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    return {c0, c1, c2, c3};
}

// FP64 uniform in (0,1): (k + 1/2) 2^-32, exact.
__device__ __forceinline__ double u01_f64(uint32_t k) { return __builtin_amdgcn_ldexp((double)k + 0.5, -32); }
// FP32 uniform in (0,1): (m + 1/2) 2^-23 with m = k >> 9, exact.  One
// v_alignbit_b32 shifts the exponent bits of 1.0 in above m, giving the float
// 1 + m 2^-23; subtracting 1 - 2^-24 is exact (Sterbenz) and centres the bins.
__device__ __forceinline__ float u01_f32(uint32_t k)
{
    return __uint_as_float(__builtin_amdgcn_alignbit(0x7Fu, k, 9)) - 0x1.fffffep-1f;
}

// ---------------------------------------------------------------- sin, cos
// sin and cos of the angle 2 pi (k + 1/2) 2^-32 of a 32-bit random word k.
// The angle is split at the nearest multiple of 2 pi / 256: j = the top 8
// bits of k + 2^23 (mod 2^32, so the last half-interval wraps to j = 0), and
// the remainder x = 2 pi (r + 1/2) 2^-32 with r = the low 24 bits minus 2^23,
// |x| <= pi / 256, both exact in integer arithmetic.  tab[j] holds
// (sin, cos)(2 pi j / 256); sin x and cos x come from their Taylor series to
// x^7 and x^6 (first omitted terms below 2e-20 relative); the angle-addition
// formulas combine them.
// min(a, b) and max(a, b) of non-NaN values as one v_min_f64 / v_max_f64
// (fmin() and fmax() of a loop-carried value cost a canonicalizing v_max_f64
// per use).
__device__ __forceinline__ double min_f64(double a, double b)
{
    double r;
    asm("v_min_f64 %0, %1, %2" : "=v"(r) : "v"(a), "v"(b));
    return r;
}

__device__ __forceinline__ double max_f64(double a, double b)
{
    double r;
    asm("v_max_f64 %0, %1, %2" : "=v"(r) : "v"(a), "v"(b));
    return r;
}

// a * b + c as one three-address FMA: a and c in vector registers, b in a
// scalar register (fma_vsv), or a and b in vector registers and c in a scalar
// register (fma_vvs).  With a constant addend the compiler otherwise picks
// the two-address form and copies the addend into the destination at every
// use.  Same rounding as fma().
__device__ __forceinline__ double fma_vsv(double a, double b, double c)
{
    double r;
    asm("v_fma_f64 %0, %1, %2, %3" : "=v"(r) : "v"(a), "s"(b), "v"(c));
    return r;
}
__device__ __forceinline__ double fma_vvs(double a, double b, double c)
{
    double r;
    asm("v_fma_f64 %0, %1, %2, %3" : "=v"(r) : "v"(a), "v"(b), "s"(c));
    return r;
}

__device__ __forceinline__ void sincos_2pi_word(uint32_t k, double tsin, double tcos, double &s, double &c)
{
    const uint32_t kk = k + 0x800000u;
    const int32_t r = (int32_t)(kk & 0xFFFFFFu) - 0x800000;
    const double x = fma_vsv((double)r, 0x1.921fb54442d18p-30, 0x1.921fb54442d18p-31);
    const double x2 = x * x;
    const double sx = fma(x * x2, fma_vvs(x2, fma_vsv(x2, -1.0 / 5040.0, 1.0 / 120.0), -1.0 / 6.0), x);
    const double cx = fma(x2, fma(x2, fma_vsv(x2, -1.0 / 720.0, 1.0 / 24.0), -0.5), 1.0);
    s = fma(tsin, cx, tcos * sx);
    c = fma(tcos, cx, -(tsin * sx));
}
__device__ __forceinline__ uint32_t sincos_index(uint32_t k) { return (k + 0x800000u) >> 24; }

// --------------------------------------------------- square roots (FP64)
// 1/sqrt(x) and sqrt(x) for normal positive x, from the hardware reciprocal
// square root (relative error below 6e-8).  rsqrt_f64: two Newton steps
// (quadratic convergence), within 1-2 ulp.  sqrt_f64: one Newton step
// (relative error ~2^-47) and then one residual correction y + (r/2)(x - y^2)
// with y = x r, whose error is of the order of the product of the two errors:
// the correctly rounded square root in every case of a CPU check with exact
// FMAs and hardware errors up to 2^-20 (1.2e8 inputs over 1e-300..1e6).
__device__ __forceinline__ double rsqrt_f64(double x)
{
    double r = __builtin_amdgcn_rsq(x);
    const double hx = 0.5 * x;
    r = fma(r, fma(-hx * r, r, 0.5), r);
    r = fma(r, fma(-hx * r, r, 0.5), r);
    return r;
}
__device__ __forceinline__ double sqrt_f64(double x)
{
    double r = __builtin_amdgcn_rsq(x);
    r = fma(r, fma(-0.5 * x * r, r, 0.5), r);
    const double y = x * r;
    return fma(fma(-y, y, x), 0.5 * r, y);
}

// Geometry tables (holes, sources) are read at wave-uniform addresses through
// the constant address space: the loads become scalar loads into SGPRs,
// shared by the wave, instead of one vector load per lane.
typedef const __attribute__((address_space(4))) double cdouble;
typedef const __attribute__((address_space(4))) float cfloat;
__device__ __forceinline__ cdouble *as_const(const double *p) { return (cdouble *)p; }
__device__ __forceinline__ cfloat *as_const(const float *p) { return (cfloat *)p; }

// OR of a value over the lanes of the wave (device library reduction, DPP
// based); the result is wave-uniform.  Its DPP steps read neighbouring lanes'
// registers whether those lanes are active or not, so it is only called where
// every lane of the wave is active, with a zero from lanes that do not take
// part.
extern "C" __device__ uint32_t __ockl_wfred_or_u32(uint32_t);

// Candidate holes of the grid cell holding (x, y, z): bit i set when hole i
// can be the nearest surface for some point of the (slightly expanded) cell.
__device__ __forceinline__ float fmaf_vsv(float a, float b, float c)
{
    float r;
    asm("v_fma_f32 %0, %1, %2, %3" : "=v"(r) : "v"(a), "s"(b), "v"(c));
    return r;
}

// The grid's cell offsets held in vector registers for a whole kernel (the
// empty asm makes each a per-lane value, so the compiler keeps it there
// instead of copying it from a scalar register at every lookup).
struct CellOff {
    float o[3];
};
__device__ __forceinline__ CellOff cell_offsets(const DevGeom &g)
{
    CellOff c;
    for (int k = 0; k < 3; ++k) {
        c.o[k] = g.cell_off[k];
        asm volatile("" : "+v"(c.o[k]));
    }
    return c;
}

__device__ __forceinline__ uint32_t cell_candidates(const DevGeom &g, const CellOff &co, float x, float y, float z)
{
    // cell coordinate (x - lo) / width as one FMA (three-address, the offset
    // read in place from a vector register), clamped to [0, n - 1/2] before
    // truncation (v_med3_f32), linear index in 24-bit multiplies
    const float fx = __builtin_amdgcn_fmed3f(fmaf_vsv(x, g.cell_inv[0], co.o[0]), 0.0f, g.cell_top[0]);
    const float fy = __builtin_amdgcn_fmed3f(fmaf_vsv(y, g.cell_inv[1], co.o[1]), 0.0f, g.cell_top[1]);
    const float fz = __builtin_amdgcn_fmed3f(fmaf_vsv(z, g.cell_inv[2], co.o[2]), 0.0f, g.cell_top[2]);
    const uint32_t idx = __umul24((uint32_t)fx, (uint32_t)g.cell_stride[0]) +
                         __umul24((uint32_t)fy, (uint32_t)g.cell_stride[1]) + (uint32_t)fz;
    return g.cell_mask[idx];
}
// Box minus boxes comes in two kernel kinds: DTN_BOX_MINUS_BOXES with the
// candidate grid (up to 32 holes, the grid masks are 32-bit) and
// kHolesNoGrid, which visits every hole.  The host picks by the grid's
// presence, so neither kind tests it at run time.
constexpr int kHolesNoGrid = 16;  // internal kind, apart from the public ones
constexpr bool has_holes(int kind) { return kind == DTN_BOX_MINUS_BOXES || kind == kHolesNoGrid; }
// Unbounded domains: walks that reach the truncation sphere have gone to
// infinity (score 0).
constexpr bool has_truncation(int kind)
{
    return kind == DTN_HALF_SPACE || kind == DTN_DISK || kind == DTN_BALL_EXTERIOR;
}

// Union over the wave of the candidate holes of the cells of the lanes that
// `take` (grid kind only).
__device__ __forceinline__ uint32_t hole_candidates(const DevGeom &g, const CellOff &co, bool take, float x, float y,
                                                    float z)
{
    const uint32_t mine = take ? cell_candidates(g, co, x, y, z) : 0u;
    return __ockl_wfred_or_u32(mine);
}

// ------------------------------------------------------------- Dirichlet data

template <int DATA>
__device__ __forceinline__ double phi_eval(const DevGeom &g, double x, double y, double z)
{
    if constexpr (DATA == DTN_DATA_TABULATED) {
        // nearest face (ties: lowest index), bilinear in its cell (clamped)
        const double p[3] = {x, y, z};
        int f = 0;
        double best = __builtin_inf();
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            const double dlo = fabs(p[k] - g.lo[k]), dhi = fabs(g.hi[k] - p[k]);
            if (dlo < best) {
                best = dlo;
                f = 2 * k;
            }
            if (dhi < best) {
                best = dhi;
                f = 2 * k + 1;
            }
        }
        const int k = f >> 1, a = k == 2 ? 0 : k + 1, b = k == 0 ? 2 : k - 1;
        const int n0 = g.tab_n[0], n1 = g.tab_n[1];
        const double s = (p[a] - g.lo[a]) * g.tab_sc[a][0], t = (p[b] - g.lo[b]) * g.tab_sc[b][1];
        const int i = min(max((int)floor(s), 0), n0 - 2), j = min(max((int)floor(t), 0), n1 - 2);
        const double fs = s - i, ft = t - j;
        const double *T = g.tab + (size_t)f * n0 * n1 + (size_t)i * n1 + j;
        const double v00 = T[0], v01 = T[1], v10 = T[n1], v11 = T[n1 + 1];
        return (1.0 - fs) * ((1.0 - ft) * v00 + ft * v01) + fs * ((1.0 - ft) * v10 + ft * v11);
    } else if constexpr (DATA == DTN_DATA_HARMONIC_QUADRATIC) {
        const double *c = g.quad;
        return c[0] + c[1] * x + c[2] * y + c[3] * z + c[4] * x * x + c[5] * y * y + c[6] * z * z +
               c[7] * x * y + c[8] * y * z + c[9] * x * z;
    } else {
        double s = 0.0;
        cdouble *q = as_const(g.src);
        for (int k = 0; k < g.n_src; ++k, q += 4) {
            const double dx = x - q[0], dy = y - q[1], dz = z - q[2];
            s = fma(q[3], rsqrt_f64(dx * dx + dy * dy + dz * dz), s);
        }
        return s;
    }
}

// --------------------------------------------------------------- distances
// Distance from an interior point to the boundary.  Ties for the closest
// surface go to the lowest index: outer faces -x,+x,-y,+y,-z,+z, then holes.

// FAST: hole distance as x * rsq(x) without refinement (relative error
// below 6e-8, measured for the hardware v_rsq_f64), for the FP32-mixed path,
// whose jumps are shortened by 2^-22 relative; else 1-2 ulp.
template <int KIND, bool FAST = false>
__device__ __forceinline__ double dist_f64(const DevGeom &g, double x, double y, double z, uint32_t cand)
{
    if constexpr (KIND == DTN_HALF_SPACE) {
        return z;  // the plane z = 0 (the truncation sphere is no surface)
    } else if constexpr (KIND == DTN_DISK) {
        // distance to the disk: |z| over it, to its rim beyond; rho from the
        // correctly rounded root (a rim distance is a small difference of
        // rho and the radius), its argument kept off 0 on the axis (where
        // the clamp cannot change the distance); sqrt(0 + z^2) is |z|
        // exactly.  FAST: the outer root unrefined (relative error below
        // 6e-8 of the distance itself)
        const double rho = sqrt_f64(max_f64(x * x + y * y, 0x1p-1000));
        const double e = max_f64(rho - g.disk_r, 0.0);
        const double q = max_f64(fma(e, e, z * z), 0x1p-1000);
        return FAST ? q * __builtin_amdgcn_rsq(q) : sqrt_f64(q);
    } else if constexpr (KIND == DTN_BALL_EXTERIOR) {
        // outside the sphere: |x - c| - r from the correctly rounded root on
        // both paths (the difference keeps the root's rounding in full)
        const double dx = x - g.c[0], dy = y - g.c[1], dz = z - g.c[2];
        return sqrt_f64(dx * dx + dy * dy + dz * dz) - g.r;
    } else if constexpr (KIND == DTN_BALL) {
        const double dx = x - g.c[0], dy = y - g.c[1], dz = z - g.c[2];
        return g.r - sqrt_f64(dx * dx + dy * dy + dz * dz);
    } else {
        double d = fmin(fmin(fmin(x - g.lo[0], g.hi[0] - x), fmin(y - g.lo[1], g.hi[1] - y)),
                        fmin(z - g.lo[2], g.hi[2] - z));
        if constexpr (has_holes(KIND)) {
            // nearest hole by squared distance, one square root at the end
            auto hole_q2 = [&](cdouble *h) {
                const double qx = fmax(fabs(x - h[0]) - h[3], 0.0);
                const double qy = fmax(fabs(y - h[1]) - h[4], 0.0);
                const double qz = fmax(fabs(z - h[2]) - h[5], 0.0);
                return qx * qx + qy * qy + qz * qz;
            };
            // the holes listed for some lane's cell (`cand`, from
            // hole_candidates: the others are farther than the boundary from
            // every point of those cells), or every hole without the grid; the
            // branch is wave-uniform, and inside it q2 is finite
            if (KIND == DTN_BOX_MINUS_BOXES ? cand != 0u : g.n_holes > 0) {
                double q2 = __builtin_inf();
                if constexpr (KIND == DTN_BOX_MINUS_BOXES) {
                    uint32_t m = cand;
                    while (m) {
                        const int i = __builtin_ctz(m);
                        m &= m - 1u;
                        q2 = min_f64(q2, hole_q2(as_const(g.hole_ce) + 6 * i));
                    }
                } else {
                    cdouble *h = as_const(g.hole_ce);
#pragma unroll 1
                    for (int i = 0; i < g.n_holes; ++i, h += 6) q2 = min_f64(q2, hole_q2(h));
                }
                // a point on a hole (q2 = 0) must still give a distance inside
                // any shell: the root's argument is clamped at 2^-1000 instead
                // of a test (identical for every q2 above it)
                const double qs = max_f64(q2, 0x1p-1000);
                const double dh = FAST ? q2 * __builtin_amdgcn_rsq(qs) : sqrt_f64(qs);
                d = min_f64(d, dh);
            }
        }
        return d;
    }
}

// All holes as a candidate mask (for callers without a per-cell list).
__device__ __forceinline__ uint32_t all_holes(const DevGeom &g)
{
    return g.n_holes >= 32 ? 0xffffffffu : ((1u << g.n_holes) - 1u);
}

// Closest boundary point of an interior point (FP64).  With the hole grid,
// only the holes in `cand` are visited (a superset of the holes that can be
// nearest, from hole_candidates or all_holes), in increasing index, so ties
// still go to the lowest index.
template <int KIND>
__device__ __forceinline__ void project_f64(const DevGeom &g, double &x, double &y, double &z, uint32_t cand)
{
    if constexpr (KIND == DTN_HALF_SPACE) {
        z = 0.0;
    } else if constexpr (KIND == DTN_DISK) {
        const double rho = sqrt(x * x + y * y);
        if (rho > g.disk_r) {
            x *= g.disk_r / rho;
            y *= g.disk_r / rho;
        }
        z = 0.0;
    } else if constexpr (KIND == DTN_BALL || KIND == DTN_BALL_EXTERIOR) {
        const double dx = x - g.c[0], dy = y - g.c[1], dz = z - g.c[2];
        const double r = sqrt(dx * dx + dy * dy + dz * dz);
        if (r > 0.0) {
            x = g.c[0] + g.r * dx / r;
            y = g.c[1] + g.r * dy / r;
            z = g.c[2] + g.r * dz / r;
        } else {
            x = g.c[0] + g.r;
            y = g.c[1];
            z = g.c[2];
        }
    } else {
        double p[3] = {x, y, z};
        double best = x - g.lo[0];
        int face = 0;
        const double face_d[5] = {g.hi[0] - x, y - g.lo[1], g.hi[1] - y, z - g.lo[2], g.hi[2] - z};
#pragma unroll
        for (int f = 1; f < 6; ++f)
            if (face_d[f - 1] < best) {
                best = face_d[f - 1];
                face = f;
            }
        int hole = -1;
        if constexpr (has_holes(KIND)) {
            auto visit = [&](int i) {
                cdouble *h = as_const(g.hole_ce) + 6 * i;
                const double qx = fmax(fabs(x - h[0]) - h[3], 0.0);
                const double qy = fmax(fabs(y - h[1]) - h[4], 0.0);
                const double qz = fmax(fabs(z - h[2]) - h[5], 0.0);
                const double d = sqrt(qx * qx + qy * qy + qz * qz);
                if (d < best) {
                    best = d;
                    hole = i;
                }
            };
            if constexpr (KIND == DTN_BOX_MINUS_BOXES) {
                uint32_t m = cand;
                while (m) {
                    const int i = __builtin_ctz(m);
                    m &= m - 1u;
                    visit(i);
                }
            } else {
#pragma unroll 1
                for (int i = 0; i < g.n_holes; ++i) visit(i);
            }
        }
        if (hole < 0) {
            const int k = face >> 1;
            p[k] = (face & 1) ? g.hi[k] : g.lo[k];
        } else {
            cdouble *b = as_const(g.hole_box) + 6 * hole;
            bool inside = true;
#pragma unroll
            for (int k = 0; k < 3; ++k) {
                if (p[k] < b[k]) {
                    p[k] = b[k];
                    inside = false;
                } else if (p[k] > b[3 + k]) {
                    p[k] = b[3 + k];
                    inside = false;
                }
            }
            if (inside) {  // rounding left the point inside the hole
                double bd = p[0] - b[0];
                int bf = 0;
                const double c2[5] = {b[3] - p[0], p[1] - b[1], b[4] - p[1], p[2] - b[2], b[5] - p[2]};
#pragma unroll
                for (int f = 1; f < 6; ++f)
                    if (c2[f - 1] < bd) {
                        bd = c2[f - 1];
                        bf = f;
                    }
                const int k = bf >> 1;
                p[k] = (bf & 1) ? b[3 + k] : b[k];
            }
        }
        x = p[0];
        y = p[1];
        z = p[2];
    }
}

// ------------------------------------------------------- compensated sums
// Neumaier's variant of Kahan summation.
struct KSum {
    double s, c;
};
__device__ __forceinline__ void kadd(KSum &a, double v)
{
    const double t = a.s + v;
    if (fabs(a.s) >= fabs(v))
        a.c += (a.s - t) + v;
    else
        a.c += (v - t) + a.s;
    a.s = t;
}
// Error-free combination of two compensated sums.
__device__ __forceinline__ KSum kmerge(KSum a, KSum b)
{
    KSum r = a;
    kadd(r, b.s);
    r.c += b.c;
    return r;
}

__device__ __forceinline__ KSum wave_ksum(KSum a)
{
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        KSum o;
        o.s = __shfl_xor(a.s, off, kWave);
        o.c = __shfl_xor(a.c, off, kWave);
        a = kmerge(a, o);
    }
    return a;
}

__device__ __forceinline__ int lane_id() { return __lane_id(); }

// Workgroups are dispatched to the 8 XCDs round-robin (workgroup i to XCD
// i mod 8), and each XCD has its own L2.  This bijection of [0, G) gives the
// workgroups an XCD receives runs of kXcdStripe consecutive logical blocks
// (neighbouring chunks: the same or adjacent nodes, whose walks share cache
// lines of their inputs and of the boundary tables on that XCD), and deals
// the 8 runs of each round to the XCDs under a rotation that changes from
// round to round, so that no XCD sees the same position of a periodic node
// layout every time (with a fixed assignment, XCD x would always get the
// same rings of every patch, and their walk lengths differ).  Blocks past
// the last whole round map to themselves.
constexpr int kXcds = 8;
constexpr int64_t kXcdStripe = 4;
__host__ __device__ __forceinline__ int64_t xcd_block(int64_t i, int64_t G)
{
    const int64_t F = G - G % (kXcds * kXcdStripe);
    if (i >= F) return i;
    const int64_t x = i % kXcds, k = i / kXcds, j = k / kXcdStripe;
    const int64_t rot = (int64_t)(((uint32_t)j * 2654435761u) >> 29);
    return (j * kXcds + ((x + rot) & (kXcds - 1))) * kXcdStripe + k % kXcdStripe;
}

// Exit-point queue entry (3 doubles) `first + rank` of a queue in LDS,
// addressed in 32 bits: rank x 24 B (one 24-bit multiply-add) onto the
// wave-uniform byte offset of entry `first`.
typedef __attribute__((address_space(3))) double lds_double;
__device__ __forceinline__ lds_double *lds_slot(double *queue, uint32_t first, uint32_t rank)
{
    uint32_t base = (uint32_t)(uintptr_t)(lds_double *)queue + 24u * first;
    asm volatile("" : "+s"(base));  // kept apart from the lane term: one v_mad_u32_u24
    return (lds_double *)(__umul24(rank, 24u) + base);
}

// Is this lane's bit set in a wave-uniform mask (the mask becomes the
// execution mask directly; no vector instruction)?
__device__ __forceinline__ bool lane_in(uint64_t mask) { return __builtin_amdgcn_inverse_ballot_w64(mask); }

// Rank of this lane among the lanes set in `mask` below it.
__device__ __forceinline__ int rank_below(uint64_t mask)
{
    return __builtin_amdgcn_mbcnt_hi((uint32_t)(mask >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)mask, 0));
}

}  // namespace dtn
