// Step 2 of the BIE-WOS method and the final potential.
//
//   k_nodes         hemisphere nodes of every patch (eq. bw85 layout on
//                   [0, theta_max] x equispaced azimuths)
//   k_solve         per patch: right-hand side of the local first-kind BIE,
//                     b_i = phi(x_i)/2 + DL_i - sum_k (Q.I)_ik u_k
//                   (eqs. bw49-bw51; DL is the double-layer integral of phi,
//                   zero on plane patches), the collocation solve K sigma = b
//                   and the propagated standard error of sigma.  FP64: LU
//                   substitution with the FP64 factors.  FP32-mixed: FP32
//                   factors, residual b - K sigma in FP64, refined.
//   k_lu32          per class, at plan time: FP32 LU with partial pivoting,
//                   blocked by 16 columns, trailing updates on MFMA
//                   (v_mfma_f32_16x16x4f32), the matrix held in LDS.
//   k_tile_sources  per tile: Neumann data at the 4x4 Gauss points (tile fit)
//   k_potential_*   u(x) = sum_q w_q [G sigma_q - dG/dn_y phi_q] (eq. bw03),
//                   direct sum, sources staged through LDS, partial sums per
//                   source chunk reduced in a fixed order.
#include <hip/hip_runtime.h>

#include <cstdio>

#include "dtn_device.h"
#include "dtn_internal.h"
#include "dtn_potential.h"

namespace dtn {

__device__ __forceinline__ void cross3(const double *a, const double *b, double *c)
{
    c[0] = a[1] * b[2] - a[2] * b[1];
    c[1] = a[2] * b[0] - a[0] * b[2];
    c[2] = a[0] * b[1] - a[1] * b[0];
}

// local (scaled by h) -> global: c + h (X t1 + Y t2 + Z n)
__device__ __forceinline__ void to_global(const dtn_patch &p, const double *t2, double X, double Y, double Z,
                                          double &gx, double &gy, double &gz)
{
    gx = p.c[0] + p.h * (X * p.t1[0] + Y * t2[0] + Z * p.n[0]);
    gy = p.c[1] + p.h * (X * p.t1[1] + Y * t2[1] + Z * p.n[1]);
    gz = p.c[2] + p.h * (X * p.t1[2] + Y * t2[2] + Z * p.n[2]);
}

__global__ __launch_bounds__(256) void k_nodes(const dtn_patch *__restrict__ patches,
                                               const int32_t *__restrict__ pclass,
                                               const DevClass *__restrict__ classes,
                                               const int64_t *__restrict__ node_off, double *__restrict__ nodes)
{
    const int pi = blockIdx.x;
    const dtn_patch p = patches[pi];
    const DevClass &cl = classes[pclass[pi]];
    double t2[3];
    cross3(p.n, p.t1, t2);
    const int64_t base = node_off[pi];
    for (int k = threadIdx.x; k < cl.n_nodes; k += blockDim.x) {
        double gx, gy, gz;
        to_global(p, t2, cl.node_tab[3 * k], cl.node_tab[3 * k + 1], cl.node_tab[3 * k + 2], gx, gy, gz);
        nodes[3 * (base + k)] = gx;
        nodes[3 * (base + k) + 1] = gy;
        nodes[3 * (base + k) + 2] = gz;
    }
}

// ------------------------------------------------------------------- solve

constexpr int kSolveBlock = 256;
constexpr int kMaxPanels = 128;
constexpr int kMaxNodes = 2048;

__device__ __forceinline__ double wave_sum(double v)
{
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, kWave);
    return v;
}

// Largest |v| over the wave; a NaN anywhere gives NaN (fmax would drop it).
__device__ __forceinline__ double wave_absmax(double v)
{
    v = fabs(v);
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        const double o = __shfl_xor(v, off, kWave);
        v = (o > v || o != o) ? o : v;
    }
    return v;
}

template <int DATA>
__global__ __launch_bounds__(kSolveBlock) void k_solve(DevGeom g, const dtn_patch *__restrict__ patches,
                                                       const int32_t *__restrict__ pclass,
                                                       const DevClass *__restrict__ classes,
                                                       const int64_t *__restrict__ node_off,
                                                       const int64_t *__restrict__ panel_off,
                                                       const double *__restrict__ node_stats, int mixed,
                                                       int max_sweeps, double *__restrict__ neumann,
                                                       double *__restrict__ neumann_se)
{
    __shared__ double u[kMaxNodes];
    __shared__ double v2[kMaxNodes];
    __shared__ double b[kMaxPanels];
    __shared__ double sol[kMaxPanels];
    __shared__ double res[kMaxPanels];
    __shared__ float f32[kMaxPanels];

    const int pi = blockIdx.x;
    const dtn_patch p = patches[pi];
    const DevClass &cl = classes[pclass[pi]];
    const int Np = cl.n_panels, Nn = cl.n_nodes;
    const int tid = threadIdx.x, lane = tid & (kWave - 1), wave = tid / kWave;
    const int nwaves = kSolveBlock / kWave;
    double t2[3];
    cross3(p.n, p.t1, t2);
    const int64_t nb = node_off[pi];
    for (int k = tid; k < Nn; k += kSolveBlock) {
        const double *s = node_stats + 4 * (nb + k);
        const double cnt = s[0];
        u[k] = s[1];
        v2[k] = cnt > 1.0 ? s[2] / ((cnt - 1.0) * cnt) : 0.0;  // SE^2 of the node mean
    }
    __syncthreads();

    // b_i = phi(x_i)/2 + DL_i - sum_k QI_ik u_k ; one wave per row
    for (int i = wave; i < Np; i += nwaves) {
        double acc = 0.0;
        const double *qi = cl.QI + (size_t)i * Nn;
        for (int k = lane; k < Nn; k += kWave) acc += qi[k] * u[k];
        double dl = 0.0;
        if (cl.curved) {
            const double *pts = cl.dl_pts + (size_t)i * cl.n_dl * 3;
            const double *w = cl.dl_w + (size_t)i * cl.n_dl;
            for (int q = lane; q < cl.n_dl; q += kWave) {
                const double wq = w[q];
                if (wq != 0.0) {
                    double gx, gy, gz;
                    to_global(p, t2, pts[3 * q], pts[3 * q + 1], pts[3 * q + 2], gx, gy, gz);
                    dl += wq * phi_eval<DATA>(g, gx, gy, gz);
                }
            }
        }
        acc = wave_sum(acc);
        dl = wave_sum(dl);
        if (lane == 0) {
            double gx, gy, gz;
            const double *x = cl.col_tab + 3 * i;
            to_global(p, t2, x[0], x[1], x[2], gx, gy, gz);
            b[i] = 0.5 * phi_eval<DATA>(g, gx, gy, gz) + dl - acc;
        }
    }
    __syncthreads();

    // K_hat y = b  (K = h K_hat, sigma = y / h); wave 0 does the substitutions
    if (wave == 0) {
        if (!mixed) {
            if (lane == 0) {
                for (int k = 0; k < Np; ++k) {
                    const int pk = cl.piv[k];
                    if (pk != k) {
                        const double t = b[k];
                        b[k] = b[pk];
                        b[pk] = t;
                    }
                }
            }
            __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
            __builtin_amdgcn_wave_barrier();
            for (int i = 0; i < Np; ++i) {  // forward, unit lower
                double a = 0.0;
                for (int j = lane; j < i; j += kWave) a += cl.LU[(size_t)i * Np + j] * b[j];
                a = wave_sum(a);
                if (lane == 0) b[i] -= a;
                __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
                __builtin_amdgcn_wave_barrier();
            }
            for (int i = Np - 1; i >= 0; --i) {  // backward
                double a = 0.0;
                for (int j = i + 1 + lane; j < Np; j += kWave) a += cl.LU[(size_t)i * Np + j] * b[j];
                a = wave_sum(a);
                if (lane == 0) b[i] = (b[i] - a) / cl.LU[(size_t)i * Np + i];
                __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
                __builtin_amdgcn_wave_barrier();
            }
            for (int i = lane; i < Np; i += kWave) sol[i] = b[i];
        } else {
            // FP32 factors + FP64 residual: y0 = 0, r = b; each sweep
            // y += LU32^-1 r, then r = b - K_hat y in FP64, until the
            // norm-wise backward error is at FP64 rounding level,
            //   |r|_inf <= Np 2^-53 (|K_hat|_inf |y|_inf + |b|_inf),
            // or max_sweeps sweeps (then, or on a non-finite residual, the
            // geometry's no-convergence bit is raised for dtn_check).  With
            // cond(K_hat) <= 64 (every supported layout) the bound is met
            // after three sweeps.
            double bmax = 0.0;
            for (int i = lane; i < Np; i += kWave) {
                sol[i] = 0.0;
                res[i] = b[i];
                const double a = fabs(b[i]);
                bmax = (a > bmax || a != a) ? a : bmax;
            }
            bmax = wave_absmax(bmax);
            const double tol = (double)Np * 0x1p-53;
            bool converged = false;
            __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
            __builtin_amdgcn_wave_barrier();
            for (int it = 0; it < max_sweeps && !converged; ++it) {
                if (lane == 0) {
                    for (int k = 0; k < Np; ++k) f32[k] = (float)res[k];
                    for (int k = 0; k < Np; ++k) {
                        const int pk = cl.piv32[k];
                        if (pk != k) {
                            const float t = f32[k];
                            f32[k] = f32[pk];
                            f32[pk] = t;
                        }
                    }
                }
                __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
                __builtin_amdgcn_wave_barrier();
                for (int i = 0; i < Np; ++i) {
                    float a = 0.0f;
                    for (int j = lane; j < i; j += kWave) a += cl.LU32[(size_t)i * Np + j] * f32[j];
#pragma unroll
                    for (int off = 32; off > 0; off >>= 1) a += __shfl_xor(a, off, kWave);
                    if (lane == 0) f32[i] -= a;
                    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
                    __builtin_amdgcn_wave_barrier();
                }
                for (int i = Np - 1; i >= 0; --i) {
                    float a = 0.0f;
                    for (int j = i + 1 + lane; j < Np; j += kWave) a += cl.LU32[(size_t)i * Np + j] * f32[j];
#pragma unroll
                    for (int off = 32; off > 0; off >>= 1) a += __shfl_xor(a, off, kWave);
                    if (lane == 0) f32[i] = (f32[i] - a) / cl.LU32[(size_t)i * Np + i];
                    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
                    __builtin_amdgcn_wave_barrier();
                }
                for (int i = lane; i < Np; i += kWave) sol[i] += (double)f32[i];
                __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
                __builtin_amdgcn_wave_barrier();
                // r = b - K_hat y in FP64
                for (int i = 0; i < Np; ++i) {
                    double a = 0.0;
                    for (int j = lane; j < Np; j += kWave) a += cl.K[(size_t)i * Np + j] * sol[j];
                    a = wave_sum(a);
                    if (lane == 0) res[i] = b[i] - a;
                }
                __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
                __builtin_amdgcn_wave_barrier();
                double rmax = 0.0, ymax = 0.0;
                for (int i = lane; i < Np; i += kWave) {
                    const double ra = fabs(res[i]), ya = fabs(sol[i]);
                    rmax = (ra > rmax || ra != ra) ? ra : rmax;
                    ymax = (ya > ymax || ya != ya) ? ya : ymax;
                }
                rmax = wave_absmax(rmax);
                ymax = wave_absmax(ymax);
                converged = rmax <= tol * (cl.k_inf * ymax + bmax);  // false on NaN
            }
            if (!converged && lane == 0) atomicOr(&g.status->flags, kFlagNoConv);
        }
    }
    __syncthreads();
    const double inv_h = 1.0 / p.h;
    const int64_t pb = panel_off[pi];
    for (int i = wave; i < Np; i += nwaves) {
        double a = 0.0;
        const double *ai = cl.A2 + (size_t)i * Nn;
        for (int k = lane; k < Nn; k += kWave) a += ai[k] * v2[k];
        a = wave_sum(a);
        if (lane == 0) {
            neumann[pb + i] = sol[i] * inv_h;
            if (neumann_se) neumann_se[pb + i] = sqrt(a) * inv_h;
        }
    }
}

// -------------------------------------------------------------- FP32 LU
// Blocked right-looking LU with partial pivoting of one class matrix (FP32,
// N <= 128, in LDS).  The trailing update A22 -= L21 U12 runs on MFMA:
// each wave owns 16x16 output tiles and issues v_mfma_f32_16x16x4f32 four
// times per 16-wide block column.
constexpr int kLuBlock = 256;

__global__ __launch_bounds__(kLuBlock) void k_lu32(DevClass *__restrict__ classes)
{
    __shared__ float A[kMaxPanels * kMaxPanels];
    __shared__ int piv[kMaxPanels];
    __shared__ float colmax[kLuBlock];
    __shared__ int colarg[kLuBlock];
    DevClass &cl = classes[blockIdx.x];
    const int N = cl.n_panels;
    const int tid = threadIdx.x;
    for (int e = tid; e < N * N; e += kLuBlock) A[e] = (float)cl.K[e];
    __syncthreads();
    const int NB = 16;
    for (int kb = 0; kb < N; kb += NB) {
        const int ke = min(N, kb + NB);
        // panel factorisation, columns kb..ke-1 (unblocked, full-row swaps)
        for (int k = kb; k < ke; ++k) {
            float best = -1.0f;
            int arg = k;
            for (int i = k + tid; i < N; i += kLuBlock) {
                const float v = fabsf(A[i * N + k]);
                if (v > best) {
                    best = v;
                    arg = i;
                }
            }
            colmax[tid] = best;
            colarg[tid] = arg;
            __syncthreads();
            if (tid == 0) {
                float bv = colmax[0];
                int ba = colarg[0];
                for (int t = 1; t < kLuBlock; ++t)
                    if (colmax[t] > bv || (colmax[t] == bv && colarg[t] < ba)) {
                        bv = colmax[t];
                        ba = colarg[t];
                    }
                piv[k] = ba;
            }
            __syncthreads();
            const int pk = piv[k];
            if (pk != k)
                for (int j = tid; j < N; j += kLuBlock) {
                    const float t = A[k * N + j];
                    A[k * N + j] = A[pk * N + j];
                    A[pk * N + j] = t;
                }
            __syncthreads();
            const float d = A[k * N + k];
            for (int i = k + 1 + tid; i < N; i += kLuBlock) A[i * N + k] /= d;
            __syncthreads();
            // update the rest of the panel columns
            for (int e = tid; e < (N - k - 1) * (ke - k - 1); e += kLuBlock) {
                const int i = k + 1 + e / (ke - k - 1);
                const int j = k + 1 + e % (ke - k - 1);
                A[i * N + j] -= A[i * N + k] * A[k * N + j];
            }
            __syncthreads();
        }
        if (ke >= N) break;
        // U12 = L11^-1 A12 (unit lower triangular solve), columns ke..N-1
        for (int j = ke + tid; j < N; j += kLuBlock)
            for (int i = kb + 1; i < ke; ++i) {
                float s = A[i * N + j];
                for (int t = kb; t < i; ++t) s -= A[i * N + t] * A[t * N + j];
                A[i * N + j] = s;
            }
        __syncthreads();
        // A22 -= L21 U12 on MFMA, 16x16 tiles, K = 16 (four k-steps of 4)
        const int lane = tid & 63, wave = tid >> 6;
        const int rows = N - ke, cols = N - ke;
        const int tr = (rows + 15) / 16, tc = (cols + 15) / 16;
        for (int tile = wave; tile < tr * tc; tile += kLuBlock / 64) {
            const int r0 = ke + 16 * (tile / tc), c0 = ke + 16 * (tile % tc);
            typedef float f4 __attribute__((ext_vector_type(4)));
            f4 acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
            for (int ks = 0; ks < 4; ++ks) {
                const int kk = kb + 4 * ks + (lane >> 4);
                const int ar = r0 + (lane & 15), bc = c0 + (lane & 15);
                const float av = (ar < N && kk < ke) ? A[ar * N + kk] : 0.0f;
                const float bv = (bc < N && kk < ke) ? A[kk * N + bc] : 0.0f;
                acc = __builtin_amdgcn_mfma_f32_16x16x4f32(av, bv, acc, 0, 0, 0);
            }
            // acc[r] holds C[row = 4 * (lane / 16) + r][col = lane % 16]
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int row = r0 + 4 * (lane >> 4) + r, col = c0 + (lane & 15);
                if (row < N && col < N) A[row * N + col] -= acc[r];
            }
        }
        __syncthreads();
    }
    for (int e = tid; e < N * N; e += kLuBlock) cl.LU32[e] = A[e];
    for (int k = tid; k < N; k += kLuBlock) cl.piv32[k] = piv[k];
}

// --------------------------------------------------------------- potential

template <int DATA>
// Four tiles per 64-thread block, 16 threads (one per Gauss point) each.
__global__ __launch_bounds__(64) void k_tile_sources(DevGeom g, const dtn_patch *__restrict__ patches,
                                                     const int32_t *__restrict__ pclass,
                                                     const DevClass *__restrict__ classes,
                                                     const int64_t *__restrict__ panel_off,
                                                     const double *__restrict__ neumann,
                                                     const int32_t *__restrict__ slot,
                                                     TileSource *__restrict__ src, int64_t n_tiles)
{
    const int64_t pi = (int64_t)blockIdx.x * 4 + threadIdx.x / 16;
    const int q = threadIdx.x % 16;
    if (pi >= n_tiles) return;
    const dtn_patch p = patches[pi];
    const DevClass &cl = classes[pclass[pi]];
    double t2[3];
    cross3(p.n, p.t1, t2);
    const double *sig = neumann + panel_off[pi];
    double s = 0.0;
    for (int i = 0; i < cl.n_panels; ++i) s += cl.fit[q * cl.n_panels + i] * sig[i];
    const double xi = cl.tile_gl[3 * q], eta = cl.tile_gl[3 * q + 1], w = cl.tile_gl[3 * q + 2] * p.h * p.h;
    TileSource o;
    to_global(p, t2, xi, eta, 0.0, o.x, o.y, o.z);
    o.nx = p.n[0];
    o.ny = p.n[1];
    o.nz = p.n[2];
    o.ws = w * s;
    o.wf = w * phi_eval<DATA>(g, o.x, o.y, o.z);
    const int64_t at = (int64_t)pi * 16 + q;
    src[slot ? (int64_t)slot[at] : at] = o;
}

constexpr int kPotBlock = 256;
constexpr int kPotChunk = 2048;
constexpr int kPotStage = 256;

__global__ __launch_bounds__(kPotBlock) void k_potential_partial(const TileSource *__restrict__ src, int64_t n_src,
                                                                 const double *__restrict__ targets, int64_t m,
                                                                 double *__restrict__ partial)
{
    __shared__ TileSource st[kPotStage];
    const int64_t t = (int64_t)blockIdx.x * kPotBlock + threadIdx.x;
    const int64_t s0 = (int64_t)blockIdx.y * kPotChunk;
    const int64_t s1 = min(n_src, s0 + kPotChunk);
    double x = 0, y = 0, z = 0;
    if (t < m) {
        x = targets[3 * t];
        y = targets[3 * t + 1];
        z = targets[3 * t + 2];
    }
    double acc = 0.0;
    for (int64_t b = s0; b < s1; b += kPotStage) {
        const int cnt = (int)min((int64_t)kPotStage, s1 - b);
        __syncthreads();
        if (threadIdx.x < cnt) st[threadIdx.x] = src[b + threadIdx.x];
        __syncthreads();
        for (int j = 0; j < cnt; ++j) {
            const TileSource &s = st[j];
            const double dx = x - s.x, dy = y - s.y, dz = z - s.z;
            const double r2 = dx * dx + dy * dy + dz * dz;
            const double ir = rsqrt(r2);
            const double ir3 = ir * ir * ir;
            acc += s.ws * ir - s.wf * (dx * s.nx + dy * s.ny + dz * s.nz) * ir3;
        }
    }
    if (t < m) partial[(size_t)blockIdx.y * m + t] = acc * (1.0 / (4.0 * M_PI));
}

__global__ __launch_bounds__(256) void k_potential_reduce(const double *__restrict__ partial, int nchunks, int64_t m,
                                                          double *__restrict__ u)
{
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= m) return;
    double s = 0.0;
    for (int c = 0; c < nchunks; ++c) s += partial[(size_t)c * m + t];
    u[t] = s;
}

// ----------------------------------------------------------------- launch

dtn_status launch_nodes(const Plan &p, double *nodes, hipStream_t s)
{
    hipLaunchKernelGGL(k_nodes, dim3((unsigned)p.patches.size()), dim3(256), 0, s, p.d_patches, p.d_patch_class,
                       p.d_classes, p.d_node_off, nodes);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return fail(DTN_E_DEVICE, std::string("dtn_patch_nodes: ") + hipGetErrorString(e));
    return DTN_OK;
}

dtn_status launch_solve(const Plan &p, const double *node_stats, int precision, double *neumann, double *neumann_se,
                        hipStream_t s)
{
    const int mixed = precision == DTN_FP32_MIXED ? 1 : 0;
    const dim3 grid((unsigned)p.patches.size());
    if (p.geom->dev.data_kind == DTN_DATA_TABULATED)
        hipLaunchKernelGGL(k_solve<DTN_DATA_TABULATED>, grid, dim3(kSolveBlock), 0, s, p.geom->dev, p.d_patches,
                           p.d_patch_class, p.d_classes, p.d_node_off, p.d_panel_off, node_stats, mixed,
                           p.max_sweeps, neumann, neumann_se);
    else if (p.geom->dev.data_kind == DTN_DATA_POINT_SOURCES)
        hipLaunchKernelGGL(k_solve<DTN_DATA_POINT_SOURCES>, grid, dim3(kSolveBlock), 0, s, p.geom->dev, p.d_patches,
                           p.d_patch_class, p.d_classes, p.d_node_off, p.d_panel_off, node_stats, mixed,
                           p.max_sweeps, neumann, neumann_se);
    else
        hipLaunchKernelGGL(k_solve<DTN_DATA_HARMONIC_QUADRATIC>, grid, dim3(kSolveBlock), 0, s, p.geom->dev,
                           p.d_patches, p.d_patch_class, p.d_classes, p.d_node_off, p.d_panel_off, node_stats, mixed,
                           p.max_sweeps, neumann, neumann_se);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return fail(DTN_E_DEVICE, std::string("dtn_patch_solve: ") + hipGetErrorString(e));
    return DTN_OK;
}

// ------------------------------------------------------- second kind
// Eqs. bw53-bw59: one block per patch, one wave per panel row computes
//   b_i = Q2_i u - sum_q s_w_iq phi(s_pts_iq) - c2_i phi(x_i)
// (the Gamma operator against the node means, phi at the regularised S
// rule's points and at the collocation point).  Flat classes: D = 0 and
// sigma = 2b; classes on a sphere: (1/2 I - D) sigma = b by substitution
// with the class's FP64 LU factors (wave 0).  The propagated SE takes
// (2 Q2)^2, or (M^-1 Q2)^2, against the node means' squared SE.  All
// scaled by 1/h.
template <int DATA>
__global__ __launch_bounds__(kSolveBlock) void k_solve2(DevGeom g, const dtn_patch *__restrict__ patches,
                                                        const int32_t *__restrict__ pclass,
                                                        const DevClass *__restrict__ classes,
                                                        const int64_t *__restrict__ node_off,
                                                        const int64_t *__restrict__ panel_off,
                                                        const double *__restrict__ node_stats,
                                                        double *__restrict__ neumann, double *__restrict__ neumann_se)
{
    __shared__ double u[kMaxNodes];
    __shared__ double v2[kMaxNodes];
    __shared__ double b[kMaxPanels];
    const int pi = blockIdx.x;
    const dtn_patch p = patches[pi];
    const DevClass &cl = classes[pclass[pi]];
    const int Np = cl.n_panels, Nn = cl.n_nodes, Ns = cl.n_s;
    const bool curved = cl.M2_LU != nullptr;
    const int tid = threadIdx.x, lane = tid & (kWave - 1), wave = tid / kWave;
    const int nwaves = kSolveBlock / kWave;
    double t2[3];
    cross3(p.n, p.t1, t2);
    const int64_t nb = node_off[pi];
    for (int k = tid; k < Nn; k += kSolveBlock) {
        const double *s = node_stats + 4 * (nb + k);
        const double cnt = s[0];
        u[k] = s[1];
        v2[k] = cnt > 1.0 ? s[2] / ((cnt - 1.0) * cnt) : 0.0;
    }
    __syncthreads();
    const double inv_h = 1.0 / p.h;
    for (int i = wave; i < Np; i += nwaves) {
        const double *q2 = cl.Q2 + (size_t)i * Nn;
        const double *a2 = curved ? cl.A2s + (size_t)i * Nn : nullptr;
        double acc = 0.0, var = 0.0, sp = 0.0;
        for (int k = lane; k < Nn; k += kWave) {
            const double w = q2[k];
            acc += w * u[k];
            var += (curved ? a2[k] : 4.0 * w * w) * v2[k];
        }
        const double *pts = cl.s_pts + (size_t)i * Ns * 3;
        const double *sw = cl.s_w + (size_t)i * Ns;
        for (int q = lane; q < Ns; q += kWave) {
            double gx, gy, gz;
            to_global(p, t2, pts[3 * q], pts[3 * q + 1], pts[3 * q + 2], gx, gy, gz);
            sp += sw[q] * phi_eval<DATA>(g, gx, gy, gz);
        }
        acc = wave_sum(acc);
        var = wave_sum(var);
        sp = wave_sum(sp);
        if (lane == 0) {
            double gx, gy, gz;
            const double *x = cl.col_tab + 3 * i;
            to_global(p, t2, x[0], x[1], x[2], gx, gy, gz);
            const double fx = phi_eval<DATA>(g, gx, gy, gz);
            b[i] = acc - sp - cl.c2[i] * fx;
            if (neumann_se) neumann_se[panel_off[pi] + i] = inv_h * sqrt(var);
        }
    }
    __syncthreads();
    if (!curved) {
        for (int i = tid; i < Np; i += kSolveBlock) neumann[panel_off[pi] + i] = 2.0 * inv_h * b[i];
        return;
    }
    if (wave == 0) {
        if (lane == 0)
            for (int k = 0; k < Np; ++k) {
                const int pk = cl.M2_piv[k];
                if (pk != k) {
                    const double t = b[k];
                    b[k] = b[pk];
                    b[pk] = t;
                }
            }
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
        __builtin_amdgcn_wave_barrier();
        for (int i = 0; i < Np; ++i) {  // forward, unit lower
            double a = 0.0;
            for (int j = lane; j < i; j += kWave) a += cl.M2_LU[(size_t)i * Np + j] * b[j];
            a = wave_sum(a);
            if (lane == 0) b[i] -= a;
            __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
            __builtin_amdgcn_wave_barrier();
        }
        for (int i = Np - 1; i >= 0; --i) {  // backward
            double a = 0.0;
            for (int j = i + 1 + lane; j < Np; j += kWave) a += cl.M2_LU[(size_t)i * Np + j] * b[j];
            a = wave_sum(a);
            if (lane == 0) b[i] = (b[i] - a) / cl.M2_LU[(size_t)i * Np + i];
            __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
            __builtin_amdgcn_wave_barrier();
        }
        for (int i = lane; i < Np; i += kWave) neumann[panel_off[pi] + i] = inv_h * b[i];
    }
}

dtn_status launch_solve2(const Plan &p, const double *node_stats, double *neumann, double *neumann_se, hipStream_t s)
{
    const dim3 grid((unsigned)p.patches.size());
    if (p.geom->dev.data_kind == DTN_DATA_TABULATED)
        hipLaunchKernelGGL(k_solve2<DTN_DATA_TABULATED>, grid, dim3(kSolveBlock), 0, s, p.geom->dev, p.d_patches,
                           p.d_patch_class, p.d_classes, p.d_node_off, p.d_panel_off, node_stats, neumann, neumann_se);
    else if (p.geom->dev.data_kind == DTN_DATA_POINT_SOURCES)
        hipLaunchKernelGGL(k_solve2<DTN_DATA_POINT_SOURCES>, grid, dim3(kSolveBlock), 0, s, p.geom->dev, p.d_patches,
                           p.d_patch_class, p.d_classes, p.d_node_off, p.d_panel_off, node_stats, neumann, neumann_se);
    else
        hipLaunchKernelGGL(k_solve2<DTN_DATA_HARMONIC_QUADRATIC>, grid, dim3(kSolveBlock), 0, s, p.geom->dev,
                           p.d_patches, p.d_patch_class, p.d_classes, p.d_node_off, p.d_panel_off, node_stats, neumann,
                           neumann_se);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return fail(DTN_E_DEVICE, std::string("dtn_patch_solve_second_kind: ") + hipGetErrorString(e));
    return DTN_OK;
}

// One wave per patch: sigma averaged over the ring-0 panels (the central
// disk, equal panel areas on a plane patch); its standard error from the
// node standard errors through the class's ring-0 row of K^-1 QI (scaled by
// 1/h like sigma); the walks spent on the patch; h.  ans [n][4].
__global__ __launch_bounds__(256) void k_answer(const dtn_patch *__restrict__ patches,
                                                const int32_t *__restrict__ pclass,
                                                const DevClass *__restrict__ classes,
                                                const int64_t *__restrict__ node_off,
                                                const int64_t *__restrict__ panel_off,
                                                const double *__restrict__ neumann,
                                                const double *__restrict__ node_stats,
                                                const int64_t *__restrict__ walks_used, int64_t n,
                                                double *__restrict__ ans)
{
    const int64_t pi = (int64_t)blockIdx.x * (blockDim.x / kWave) + threadIdx.x / kWave;
    if (pi >= n) return;
    const int lane = threadIdx.x & (kWave - 1);
    const DevClass &cl = classes[pclass[pi]];
    const double h = patches[pi].h;
    const int64_t nb = node_off[pi], pb = panel_off[pi];
    double v = 0.0, w = 0.0;
    for (int k = lane; k < cl.n_nodes; k += kWave) {
        const double *st = node_stats + 4 * (nb + k);
        const double se2 = st[0] > 1.0 ? st[2] / ((st[0] - 1.0) * st[0]) : 0.0;
        const double a = cl.ans_row[k];
        v += a * a * se2;
        w += (double)walks_used[nb + k];
    }
    double m = 0.0;
    for (int i = lane; i < cl.n_sectors; i += kWave) m += neumann[pb + i];
    v = wave_sum(v);
    w = wave_sum(w);
    m = wave_sum(m);
    if (lane == 0) {
        ans[4 * pi] = m / cl.n_sectors;
        ans[4 * pi + 1] = sqrt(v) / h;
        ans[4 * pi + 2] = w;
        ans[4 * pi + 3] = h;
    }
}

dtn_status launch_answer(const Plan &p, const double *neumann, const double *node_stats, const int64_t *walks_used,
                         double *ans, hipStream_t s)
{
    const int64_t n = (int64_t)p.patches.size();
    if (n == 0) return DTN_OK;
    hipLaunchKernelGGL(k_answer, dim3((unsigned)((n + 3) / 4)), dim3(256), 0, s, p.d_patches, p.d_patch_class,
                       p.d_classes, p.d_node_off, p.d_panel_off, neumann, node_stats, walks_used, n, ans);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return fail(DTN_E_DEVICE, std::string("answer: ") + hipGetErrorString(e));
    return DTN_OK;
}

// Per-node walk identity of a batch of queries: every node of patch p gets
// its query's Philox key and squared SE target, and stream id = its index
// within the query (sid0[p] + node index in the patch).
__global__ __launch_bounds__(256) void k_node_ids(int64_t n_patches, int nn, const uint64_t *__restrict__ pseed,
                                                  const uint32_t *__restrict__ psid0,
                                                  const double *__restrict__ pse2, uint64_t *__restrict__ nseed,
                                                  uint32_t *__restrict__ nsid, double *__restrict__ nse2)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n_patches * nn) return;
    const int64_t p = i / nn;
    nseed[i] = pseed[p];
    nsid[i] = psid0[p] + (uint32_t)(i - p * nn);
    nse2[i] = pse2[p];
}

dtn_status launch_node_ids(int64_t n_patches, int nn, const uint64_t *pseed, const uint32_t *psid0,
                           const double *pse2, uint64_t *nseed, uint32_t *nsid, double *nse2, hipStream_t s)
{
    const int64_t n = n_patches * nn;
    if (n == 0) return DTN_OK;
    hipLaunchKernelGGL(k_node_ids, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, n_patches, nn, pseed, psid0,
                       pse2, nseed, nsid, nse2);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return fail(DTN_E_DEVICE, std::string("node ids: ") + hipGetErrorString(e));
    return DTN_OK;
}

dtn_status launch_lu32(const Plan &p, hipStream_t s)
{
    hipLaunchKernelGGL(k_lu32, dim3((unsigned)p.classes.size()), dim3(kLuBlock), 0, s, p.d_classes);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return fail(DTN_E_DEVICE, std::string("dtn_create_plan (lu32): ") + hipGetErrorString(e));
    return DTN_OK;
}

dtn_status launch_tile_sources(const Plan &p, const double *neumann, const int32_t *slot, TileSource *src,
                               hipStream_t s)
{
    const int64_t n = (int64_t)p.patches.size();
    const dim3 grid((unsigned)((n + 3) / 4));
    if (p.geom->dev.data_kind == DTN_DATA_TABULATED)
        hipLaunchKernelGGL(k_tile_sources<DTN_DATA_TABULATED>, grid, dim3(64), 0, s, p.geom->dev, p.d_patches,
                           p.d_patch_class, p.d_classes, p.d_panel_off, neumann, slot, src, n);
    else if (p.geom->dev.data_kind == DTN_DATA_POINT_SOURCES)
        hipLaunchKernelGGL(k_tile_sources<DTN_DATA_POINT_SOURCES>, grid, dim3(64), 0, s, p.geom->dev, p.d_patches,
                           p.d_patch_class, p.d_classes, p.d_panel_off, neumann, slot, src, n);
    else
        hipLaunchKernelGGL(k_tile_sources<DTN_DATA_HARMONIC_QUADRATIC>, grid, dim3(64), 0, s, p.geom->dev,
                           p.d_patches, p.d_patch_class, p.d_classes, p.d_panel_off, neumann, slot, src, n);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return fail(DTN_E_DEVICE, std::string("tile sources: ") + hipGetErrorString(e));
    return DTN_OK;
}

dtn_status launch_potential(const Plan &p, const double *neumann, const double *targets, int64_t m, double *u_out,
                            hipStream_t s)
{
    if (m == 0) return DTN_OK;
    const int64_t n_src = (int64_t)p.patches.size() * 16;
    const int nchunks = (int)((n_src + kPotChunk - 1) / kPotChunk);
    const size_t bytes = sizeof(TileSource) * (size_t)n_src + sizeof(double) * (size_t)nchunks * (size_t)m;
    char *scratch = nullptr;
    hipError_t e = hipMallocAsync((void **)&scratch, bytes, s);
    if (e != hipSuccess) return fail(DTN_E_OOM, std::string("dtn_potential: ") + hipGetErrorString(e));
    TileSource *src = (TileSource *)scratch;
    double *partial = (double *)(scratch + sizeof(TileSource) * (size_t)n_src);
    const dtn_status st = launch_tile_sources(p, neumann, nullptr, src, s);
    if (st != DTN_OK) {
        (void)hipFreeAsync(scratch, s);
        return st;
    }
    hipLaunchKernelGGL(k_potential_partial, dim3((unsigned)((m + kPotBlock - 1) / kPotBlock), (unsigned)nchunks),
                       dim3(kPotBlock), 0, s, src, n_src, targets, m, partial);
    hipLaunchKernelGGL(k_potential_reduce, dim3((unsigned)((m + 255) / 256)), dim3(256), 0, s, partial, nchunks, m,
                       u_out);
    e = hipGetLastError();
    if (e == hipSuccess) e = hipFreeAsync(scratch, s);
    if (e != hipSuccess) return fail(DTN_E_DEVICE, std::string("dtn_potential: ") + hipGetErrorString(e));
    return DTN_OK;
}

}  // namespace dtn
