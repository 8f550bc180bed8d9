// Walk-on-spheres kernels: step 1 of the BIE-WOS method.
//
// u(y) = E[phi(X_tau)] (Sec. 2, eq. bw13), sampled by walk on spheres with an
// epsilon absorbing shell (Sec. 2, after Fig. fig_wos): from x jump to a
// uniform point of the sphere of radius dist(x, boundary); stop once the
// distance is below eps and record phi at the closest boundary point.  The
// node estimate is the mean of the recorded values (Sec. 5.1.2, eq. bw87);
// the kernels also keep the sum of squares for the standard error.
//
// Work decomposition (all on the device, no host round trip):
//   k_wos_plan      one workgroup: total walks -> chunk size C, per-point
//                   chunk counts and their exclusive scan (chunk offsets);
//                   for many points the same in three launches over
//                   segments (k_plan_sum, k_plan_count, k_plan_write)
//   k_wos_walk      one wave per chunk (point, walk range of <= C walks); the
//                   wave runs its walks with refill: a lane whose walk ends takes
//                   the next walk of the chunk, so lanes do not idle behind
//                   long walks.  Absorbed positions are queued in LDS and
//                   projected and scored 64 at a time by the whole wave, so
//                   that code runs with full lanes.  Which lanes hold a walk is
//                   a wave-uniform mask; jumps and capped walks are counted
//                   from it on the scalar unit.  Per-lane compensated FP64
//                   sums are reduced across the wave and written per chunk.
//   k_wos_finalize  per point: merge its chunks in chunk order (fixed
//                   order, so results do not depend on which wave ran which
//                   chunk), write (count, mean, M2, steps) and capped count.
//
// Unbounded domains (half space, exterior of a disk or a ball): a walk that reaches the
// truncation sphere has gone to infinity and scores 0 (Sec. 5.1.3); the
// sphere is tested before the shell.  Such a walk is queued with z = +inf
// (every other queued position is finite).
//
// Randomness: walk k of a point with stream id s draws Philox4x32-10 block
// (k lo, k hi, j, s) for its steps 2j and 2j+1 (words 0,1 then 2,3).  New
// walks start on even wave iterations only, so every live lane is at the
// same step parity and the Philox call is wave-uniform (no divergence).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdio>
#include <map>
#include <mutex>
#include <string>

#include "dtn_device.h"
#include "dtn_internal.h"

namespace dtn {

struct ChunkPartial {
    double s1, c1, s2, c2;
    unsigned long long steps, capped;
};

constexpr int kPlanThreads = 1024;
constexpr int kWalkBlock = 256;  // 4 waves
constexpr int kQueue = 128;      // exit-point queue slots per wave

__device__ __forceinline__ int64_t uniform64(int64_t v)
{
    const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)(uint64_t)v);
    const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)((uint64_t)v >> 32));
    return (int64_t)(((uint64_t)hi << 32) | lo);
}

__device__ __forceinline__ void wave_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
}

// ----------------------------------------------------------------- planning
// meta[0] = chunk size C, meta[1] = total chunks.
__global__ __launch_bounds__(kPlanThreads) void k_wos_plan(const int64_t *__restrict__ walks, int64_t n,
                                                           int64_t target_chunks, int64_t c_min,
                                                           int64_t *__restrict__ chunk_off,
                                                           int64_t *__restrict__ meta)
{
    __shared__ int64_t red[kPlanThreads];
    const int t = threadIdx.x;
    int64_t tot = 0;
    for (int64_t i = t; i < n; i += kPlanThreads) tot += max(walks[i], (int64_t)0);
    red[t] = tot;
    __syncthreads();
    for (int s = kPlanThreads / 2; s > 0; s >>= 1) {
        if (t < s) red[t] += red[t + s];
        __syncthreads();
    }
    const int64_t total_walks = red[0];
    __syncthreads();
    const int64_t C = max(c_min, (total_walks + target_chunks - 1) / target_chunks);
    // contiguous segments per thread, then a block scan of segment sums
    const int64_t L = (n + kPlanThreads - 1) / kPlanThreads;
    const int64_t b = min(n, (int64_t)t * L), e = min(n, b + L);
    int64_t seg = 0;
    for (int64_t i = b; i < e; ++i) seg += (max(walks[i], (int64_t)0) + C - 1) / C;
    red[t] = seg;
    __syncthreads();
    for (int s = 1; s < kPlanThreads; s <<= 1) {  // Hillis-Steele inclusive scan
        const int64_t v = (t >= s) ? red[t - s] : 0;
        __syncthreads();
        red[t] += v;
        __syncthreads();
    }
    int64_t run = red[t] - seg;
    for (int64_t i = b; i < e; ++i) {
        chunk_off[i] = run;
        run += (max(walks[i], (int64_t)0) + C - 1) / C;
    }
    if (t == kPlanThreads - 1) {
        chunk_off[n] = red[t];
        meta[0] = C;
        meta[1] = red[t];
    }
}

// Multi-block planning (many points): B segments of L consecutive points.
//   k_plan_sum    per segment: sum of its walk counts -> part[b]
//   k_plan_count  per segment: C from the sum of part[] (every block
//                 computes the same value), the segment's chunk count ->
//                 cnt[b]; block 0 writes meta[0] = C
//   k_plan_write  per segment: base = sum of cnt[j < b], a block scan of the
//                 points' chunk counts -> chunk_off; the last block writes
//                 chunk_off[n] and meta[1]
// Same integers as k_wos_plan (every value is an exact integer sum).
constexpr int kSegThreads = 256;

__device__ __forceinline__ int64_t block_sum_i64(int64_t v, int64_t *red)
{
    const int t = threadIdx.x;
    red[t] = v;
    __syncthreads();
    for (int s = kSegThreads / 2; s > 0; s >>= 1) {
        if (t < s) red[t] += red[t + s];
        __syncthreads();
    }
    const int64_t r = red[0];
    __syncthreads();
    return r;
}

__global__ __launch_bounds__(kSegThreads) void k_plan_sum(const int64_t *__restrict__ walks, int64_t n, int64_t L,
                                                          int64_t *__restrict__ part)
{
    __shared__ int64_t red[kSegThreads];
    const int64_t b0 = (int64_t)blockIdx.x * L, b1 = min(n, b0 + L);
    int64_t s = 0;
    for (int64_t i = b0 + threadIdx.x; i < b1; i += kSegThreads) s += max(walks[i], (int64_t)0);
    s = block_sum_i64(s, red);
    if (threadIdx.x == 0) part[blockIdx.x] = s;
}

__device__ __forceinline__ int64_t plan_chunk(const int64_t *__restrict__ part, int nb, int64_t target_chunks,
                                              int64_t c_min, int64_t *red)
{
    int64_t s = 0;
    for (int j = threadIdx.x; j < nb; j += kSegThreads) s += part[j];
    const int64_t total = block_sum_i64(s, red);
    return max(c_min, (total + target_chunks - 1) / target_chunks);
}

__global__ __launch_bounds__(kSegThreads) void k_plan_count(const int64_t *__restrict__ walks, int64_t n, int64_t L,
                                                            const int64_t *__restrict__ part, int nb,
                                                            int64_t target_chunks, int64_t c_min,
                                                            int64_t *__restrict__ cnt, int64_t *__restrict__ meta)
{
    __shared__ int64_t red[kSegThreads];
    const int64_t C = plan_chunk(part, nb, target_chunks, c_min, red);
    const int64_t b0 = (int64_t)blockIdx.x * L, b1 = min(n, b0 + L);
    int64_t s = 0;
    for (int64_t i = b0 + threadIdx.x; i < b1; i += kSegThreads) s += (max(walks[i], (int64_t)0) + C - 1) / C;
    s = block_sum_i64(s, red);
    if (threadIdx.x == 0) {
        cnt[blockIdx.x] = s;
        if (blockIdx.x == 0) meta[0] = C;
    }
}

__global__ __launch_bounds__(kSegThreads) void k_plan_write(const int64_t *__restrict__ walks, int64_t n, int64_t L,
                                                            const int64_t *__restrict__ cnt,
                                                            int64_t *__restrict__ chunk_off,
                                                            int64_t *__restrict__ meta)
{
    __shared__ int64_t red[kSegThreads];
    const int t = threadIdx.x;
    const int64_t C = meta[0];
    int64_t s = 0;
    for (int j = t; j < (int)blockIdx.x; j += kSegThreads) s += cnt[j];
    const int64_t base = block_sum_i64(s, red);
    // contiguous runs per thread, then a scan of the run sums
    const int64_t b0 = (int64_t)blockIdx.x * L, b1 = min(n, b0 + L);
    const int64_t R = (b1 - b0 + kSegThreads - 1) / kSegThreads;
    const int64_t r0 = min(b1, b0 + t * R), r1 = min(b1, r0 + R);
    int64_t run = 0;
    for (int64_t i = r0; i < r1; ++i) run += (max(walks[i], (int64_t)0) + C - 1) / C;
    red[t] = run;
    __syncthreads();
    for (int o = 1; o < kSegThreads; o <<= 1) {  // Hillis-Steele inclusive scan
        const int64_t v = t >= o ? red[t - o] : 0;
        __syncthreads();
        red[t] += v;
        __syncthreads();
    }
    int64_t off = base + red[t] - run;
    for (int64_t i = r0; i < r1; ++i) {
        chunk_off[i] = off;
        off += (max(walks[i], (int64_t)0) + C - 1) / C;
    }
    if (blockIdx.x == gridDim.x - 1 && t == kSegThreads - 1) {
        chunk_off[n] = base + red[t];
        meta[1] = base + red[t];
    }
}

// ---------------------------------------------------------------- the walks

// Score of a queued exit position: phi at its closest boundary point, or 0
// for a walk gone to infinity (queued with z = +inf).
template <int KIND, int DATA>
__device__ __forceinline__ double exit_score(const DevGeom &g, double px, double py, double pz, uint32_t pc)
{
    const bool gone = has_truncation(KIND) && pz == __builtin_inf();
    project_f64<KIND>(g, px, py, pz, pc);
    const double f = phi_eval<DATA>(g, px, py, pz);
    return gone ? 0.0 : f;
}

template <int KIND, int DATA, int PREC>
__global__ __launch_bounds__(kWalkBlock) void k_wos_walk(DevGeom g, const double *__restrict__ pts,
                                                         const int64_t *__restrict__ walks,
                                                         const int64_t *__restrict__ walk_begin,
                                                         const uint32_t *__restrict__ stream_id, uint64_t seed,
                                                         const uint64_t *__restrict__ node_seed,
                                                         const int64_t *__restrict__ chunk_off,
                                                         const int64_t *__restrict__ meta, int64_t n,
                                                         ChunkPartial *__restrict__ out)
{
    __shared__ double queue[kWalkBlock / kWave][kQueue * 3];
    __shared__ double sc_tab[256][2];  // (sin, cos) of 2 pi j / 256, FP64 path
    if constexpr (PREC == DTN_FP64) {
        for (int i = threadIdx.x; i < 512; i += kWalkBlock) (&sc_tab[0][0])[i] = g.sincos[i];
        __syncthreads();
    }
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
    double *q = queue[wave];
    const int lane = lane_id();
    // one chunk per wave; chunk size and count are wave-uniform (SGPRs)
    const int64_t C = uniform64(meta[0]);
    const int64_t total = uniform64(meta[1]);
    const int64_t chunk = xcd_block(blockIdx.x, gridDim.x) * (kWalkBlock / kWave) + wave;
    if (chunk >= total) return;
    const double eps = g.eps;
    {
        // point owning this chunk: largest i with chunk_off[i] <= chunk
        int64_t lo = 0, hi = n;
        while (hi - lo > 1) {
            const int64_t mid = (lo + hi) >> 1;
            if (chunk_off[mid] <= chunk) lo = mid; else hi = mid;
        }
        const int64_t node = lo;
        const int64_t wnode = max(walks[node], (int64_t)0);
        const int64_t w_lo = (chunk - chunk_off[node]) * C;
        const int64_t w_hi = min(wnode, w_lo + C);
        const int64_t wb = walk_begin ? walk_begin[node] : 0;
        const uint32_t sid = stream_id ? stream_id[node] : (uint32_t)node;
        const uint64_t key = node_seed ? (uint64_t)uniform64((int64_t)node_seed[node]) : seed;
        const uint32_t k0 = (uint32_t)key, k1 = (uint32_t)(key >> 32);
        const double y0 = pts[3 * node], y1 = pts[3 * node + 1], y2 = pts[3 * node + 2];
        double sx = y0, sy = y1, sz = y2;
        project_f64<KIND>(g, sx, sy, sz, all_holes(g));
        const double shift = phi_eval<DATA>(g, sx, sy, sz);

        const CellOff co = KIND == DTN_BOX_MINUS_BOXES ? cell_offsets(g) : CellOff{};
        // lane state; which lanes hold a walk is the wave-uniform mask
        // `wmask` (scalar registers): lane predicates come from it with no
        // vector instruction, and ballots of compares fold into it
        uint64_t wmask = 0;
        uint64_t walk = 0;
        double x = y0, y = y1, z = y2;
        uint32_t nstep = 0;
        uint32_t r2 = 0, r3 = 0;
        KSum s1{0.0, 0.0}, s2{0.0, 0.0};
        // jumps and capped walks of the chunk, counted from the masks
        // (wave-uniform): a lane jumps when it walks and does not stop, a
        // stopping lane is capped when it is not inside the shell
        uint64_t steps = 0, capped = 0;
        // box minus holes: wave iterations and hole distances computed
        // (scalar counters, added up when counting is on)
        uint64_t n_iters = 0, n_visits = 0;
        int64_t next = w_lo;  // wave-uniform: next walk to hand out
        int qn = 0;           // wave-uniform: queued exit points
        // step cap (a walk's step count is 32-bit; geometries with a larger
        // cap are rejected at creation)
        const uint32_t cap = (uint32_t)min(g.max_steps, (int64_t)0xffffffff);
        // Hard bound on wave iterations: every walk ends within cap + 2
        // iterations of its start and a lane runs at most ceil(C/64) walks.
        // Saturating, so that no cap or chunk size makes the product wrap.
        const uint64_t per_walk = 2ull * ((uint64_t)cap + 4ull);
        const uint64_t per_lane = (uint64_t)((w_hi - w_lo + kWave - 1) / kWave + 1);
        const uint64_t it_max = per_lane > ~0ull / per_walk ? ~0ull : per_walk * per_lane;

        // Where a walk's exit is tested, by measurement per kernel: right
        // after the jump that reached its position (the distance taken
        // there), so that a walk of S steps holds its lane S iterations, not
        // S + 1 (FP64 walks and box-with-holes walks: 0.6 % and 1 % faster),
        // or at the top of the next iteration, where the distance runs
        // beside the direction (FP32-mixed walks on the other kinds: their
        // hardware sin/cos overlaps the FP64 distance there, 4 % faster).
        // With the test after the jump every walk starts at the chunk's
        // point, so the start's distance and exit test are taken once.
        constexpr bool kExitAfterJump = PREC == DTN_FP64 || KIND == DTN_BOX_MINUS_BOXES;
        double d = 0.0;
        bool start_ends = false;
        if constexpr (kExitAfterJump) {
            uint32_t cand0 = 0;
            if constexpr (KIND == DTN_BOX_MINUS_BOXES)
                cand0 = hole_candidates(g, co, true, (float)y0, (float)y1, (float)y2);
            d = dist_f64<KIND, PREC != DTN_FP64>(g, y0, y1, y2, cand0);
            if constexpr (has_holes(KIND)) {
                ++n_iters;
                n_visits += KIND == DTN_BOX_MINUS_BOXES ? (uint64_t)__builtin_popcount(cand0) : (uint64_t)g.n_holes;
            }
            bool start_gone = false;
            if constexpr (has_truncation(KIND)) {
                const double ex = y0 - g.c[0], ey = y1 - g.c[1], ez = y2 - g.c[2];
                start_gone = ex * ex + ey * ey + ez * ez >= g.trunc_r * g.trunc_r;
            }
            // every lane computed the same start; the ballot makes that
            // wave-uniform for the compiler
            start_ends = __builtin_amdgcn_ballot_w64(d < eps || start_gone) != 0 || cap == 0u;
        }
        const double d0 = d;

        for (uint64_t it = 0; it < it_max; ++it) {
            uint32_t w1, w2;  // this step's two random words
            uint64_t fm0 = 0;  // walks handed out now that end at their start (exit after the jump)
            if ((it & 1ull) == 0ull) {
                const uint64_t want = ~wmask;
                if (want) {
                    // the idle lanes take the next walks in lane order while
                    // any are left (ballot of the plain compare, masked in
                    // scalar registers)
                    const int64_t mine = next + rank_below(want);
                    const uint64_t sm = want & __builtin_amdgcn_ballot_w64(mine < w_hi);
                    if (lane_in(sm)) {
                        walk = (uint64_t)(wb + mine);
                        x = y0;
                        y = y1;
                        z = y2;
                        d = d0;
                        nstep = 0;
                    }
                    wmask |= sm;
                    next += __popcll(want);
                    if constexpr (kExitAfterJump) fm0 = start_ends ? sm : 0;
                }
                if (wmask == 0) break;
                const Philox4 r = philox4x32_10((uint32_t)walk, (uint32_t)(walk >> 32), nstep >> 1, sid, k0, k1);
                w1 = r.x;
                w2 = r.y;
                r2 = r.z;
                r3 = r.w;
            } else {
                w1 = r2;
                w2 = r3;
            }
            // The distance at the lanes' positions and the exit tests: inside
            // the shell, beyond the truncation sphere, at the step cap (the
            // last returned).  Distance and epsilon test in FP64 on both paths
            // (an FP32 distance would need an FP64 recheck inside a rounding
            // band around the shell, which some lane of a wave needs at almost
            // every step, and a shrunken jump everywhere).  Every lane
            // computes it (an idle lane's point is its last one, inside the
            // domain); only the walking lanes' results are used.
            uint64_t in_shell = 0, gone = 0;
            const auto exit_tests = [&]() {
                // candidate holes of the walking lanes' cells (whole wave active here)
                uint32_t cand = 0;
                if constexpr (KIND == DTN_BOX_MINUS_BOXES)
                    cand = hole_candidates(g, co, lane_in(wmask), (float)x, (float)y, (float)z);
                if constexpr (has_holes(KIND)) {
                    ++n_iters;
                    n_visits += KIND == DTN_BOX_MINUS_BOXES ? (uint64_t)__builtin_popcount(cand) : (uint64_t)g.n_holes;
                }
                d = dist_f64<KIND, PREC != DTN_FP64>(g, x, y, z, cand);
                in_shell = __builtin_amdgcn_ballot_w64(d < eps);
                if constexpr (has_truncation(KIND)) {
                    const double ex = x - g.c[0], ey = y - g.c[1], ez = z - g.c[2];
                    gone = __builtin_amdgcn_ballot_w64(ex * ex + ey * ey + ez * ez >= g.trunc_r * g.trunc_r);
                }
                return __builtin_amdgcn_ballot_w64(nstep >= cap);
            };
            uint64_t fm = 0;  // walks that end in this iteration
            if constexpr (!kExitAfterJump) {
                const uint64_t at_cap = exit_tests();
                fm = wmask & (in_shell | gone | at_cap);
            }
            // the walking lanes that go on jump by d (the distance at their
            // position, at least eps)
            const uint64_t jm = wmask & ~(kExitAfterJump ? fm0 : fm);
            steps += (uint64_t)__popcll(jm);
            if (lane_in(jm)) {
                if constexpr (PREC == DTN_FP64) {
                    const double u1d = u01_f64(w1);
                    const double cz = 1.0 - 2.0 * u1d;
                    const double sr = 2.0 * sqrt_f64(u1d * (1.0 - u1d));
                    const uint32_t j = sincos_index(w2);
                    double sn, cs;
                    sincos_2pi_word(w2, sc_tab[j][0], sc_tab[j][1], sn, cs);
                    x += d * (sr * cs);
                    y += d * (sr * sn);
                    z += d * cz;
                } else {
                    // FP32 direction: uniforms, square root and the
                    // hardware sin/cos (revolution input); |omega| = 1
                    // within three FP32 roundings, so the jump is
                    // shortened by 2^-22 to stay inside the ball
                    const float u1f = u01_f32(w1), u2f = u01_f32(w2);
                    const float cz = 1.0f - 2.0f * u1f;
                    const float sr = 2.0f * __builtin_amdgcn_sqrtf(u1f * (1.0f - u1f));
                    const float cs = __builtin_amdgcn_cosf(u2f);  // cos(2 pi u2)
                    const float sn = __builtin_amdgcn_sinf(u2f);  // sin(2 pi u2)
                    const double dj = d * (1.0 - 0x1p-22);
                    x += dj * (double)(sr * cs);
                    y += dj * (double)(sr * sn);
                    z += dj * (double)cz;
                }
                ++nstep;
            }
            if constexpr (kExitAfterJump) {
                const uint64_t at_cap = exit_tests();
                fm = (jm & (in_shell | gone | at_cap)) | fm0;
            }
            capped += (uint64_t)__popcll(fm & ~(in_shell | gone));
            if (fm) {
                if (lane_in(fm)) {
                    // 32-bit LDS address: lane rank x 24 B onto a scalar base
                    lds_double *e = lds_slot(q, (uint32_t)qn, (uint32_t)rank_below(fm));
                    e[0] = x;
                    e[1] = y;
                    e[2] = (has_truncation(KIND) && lane_in(gone)) ? __builtin_inf() : z;
                }
                wmask &= ~fm;
                qn += __popcll(fm);
                if (qn >= kWave) {
                    wave_sync();
                    double px = q[3 * lane], py = q[3 * lane + 1], pz = q[3 * lane + 2];
                    uint32_t pc = 0;  // candidate holes of the 64 queued points (whole wave active)
                    if constexpr (KIND == DTN_BOX_MINUS_BOXES)
                        pc = hole_candidates(g, co, true, (float)px, (float)py, (float)pz);
                    const double v = exit_score<KIND, DATA>(g, px, py, pz, pc) - shift;
                    kadd(s1, v);
                    kadd(s2, v * v);
                    const int rest = qn - kWave;
                    double a0 = 0, a1 = 0, a2 = 0;
                    if (lane < rest) {
                        a0 = q[3 * (kWave + lane)];
                        a1 = q[3 * (kWave + lane) + 1];
                        a2 = q[3 * (kWave + lane) + 2];
                    }
                    wave_sync();
                    if (lane < rest) {
                        q[3 * lane] = a0;
                        q[3 * lane + 1] = a1;
                        q[3 * lane + 2] = a2;
                    }
                    wave_sync();
                    qn = rest;
                }
            }
        }
        // walks still running or never started when the bound ends the loop
        // (not reached under the bound above) are counted as capped, so a
        // short sum is never silent
        capped += (uint64_t)__popcll(wmask) + (uint64_t)(next < w_hi ? w_hi - next : 0);
        // score what is left in the queue
        wave_sync();
        {
            const bool has = lane < qn;
            double px = has ? q[3 * lane] : 0.0, py = has ? q[3 * lane + 1] : 0.0, pz = has ? q[3 * lane + 2] : 0.0;
            uint32_t pc = 0;
            if constexpr (KIND == DTN_BOX_MINUS_BOXES)
                pc = hole_candidates(g, co, has, (float)px, (float)py, (float)pz);
            if (has) {
                const double v = exit_score<KIND, DATA>(g, px, py, pz, pc) - shift;
                kadd(s1, v);
                kadd(s2, v * v);
            }
        }
        wave_sync();
        const KSum t1 = wave_ksum(s1);
        const KSum t2 = wave_ksum(s2);
        const unsigned long long ts = steps;
        const unsigned long long tc = capped;
        if constexpr (has_holes(KIND)) {
            // two device-wide atomics per chunk serialise on one address:
            // only in the counting mode dtn_walk_counters switches on
            if (g.count_walks && lane == 0) {
                atomicAdd(&g.status->iters, (unsigned long long)n_iters);
                atomicAdd(&g.status->visits, (unsigned long long)n_visits);
            }
        }
        if (lane == 0) {
            ChunkPartial p;
            p.s1 = t1.s;
            p.c1 = t1.c;
            p.s2 = t2.s;
            p.c2 = t2.c;
            p.steps = ts;
            p.capped = tc;
            out[chunk] = p;
        }
    }
}

// --------------------------------------------------------------- finalize

template <int KIND, int DATA>
__global__ __launch_bounds__(256) void k_wos_finalize(DevGeom g, const double *__restrict__ pts,
                                                      const int64_t *__restrict__ walks, int64_t n,
                                                      const int64_t *__restrict__ chunk_off,
                                                      const ChunkPartial *__restrict__ part,
                                                      double *__restrict__ stats, int64_t *__restrict__ capped)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    KSum s1{0.0, 0.0}, s2{0.0, 0.0};
    unsigned long long st = 0, cp = 0;
    for (int64_t c = chunk_off[i]; c < chunk_off[i + 1]; ++c) {
        const ChunkPartial p = part[c];
        s1 = kmerge(s1, KSum{p.s1, p.c1});
        s2 = kmerge(s2, KSum{p.s2, p.c2});
        st += p.steps;
        cp += p.capped;
    }
    const int64_t w = max(walks[i], (int64_t)0);
    double sx = pts[3 * i], sy = pts[3 * i + 1], sz = pts[3 * i + 2];
    project_f64<KIND>(g, sx, sy, sz, all_holes(g));
    const double shift = phi_eval<DATA>(g, sx, sy, sz);
    const double cnt = (double)w;
    const double S1 = s1.s + s1.c, S2 = s2.s + s2.c;
    double mean = 0.0, m2 = 0.0;
    if (w > 0) {
        mean = shift + S1 / cnt;
        m2 = S2 - S1 * S1 / cnt;
        if (m2 < 0.0) m2 = 0.0;
    }
    stats[4 * i] = cnt;
    stats[4 * i + 1] = mean;
    stats[4 * i + 2] = m2;
    stats[4 * i + 3] = (double)st;
    if (capped) capped[i] = (int64_t)cp;
    if (cp != 0) atomicOr(&g.status->flags, kFlagCapped);  // reported by dtn_check
}

// ----------------------------------------------------------------- launch

int device_cus()
{
    static thread_local int cached_dev = -1, cached_cus = 0;
    int dev = 0;
    (void)hipGetDevice(&dev);
    if (dev != cached_dev) {
        hipDeviceProp_t prop;
        cached_cus = hipGetDeviceProperties(&prop, dev) == hipSuccess ? prop.multiProcessorCount : 256;
        cached_dev = dev;
    }
    return cached_cus > 0 ? cached_cus : 256;
}

namespace {

// Launch shape and scratch of one walk launch over n points: the chunk
// target (`oversub` chunks per resident wave, 4 SIMDs x 8 waves per CU), the
// bound on the chunk count (total chunks <= sum(walks)/C + n <= target + n),
// the multi-block plan over nb segments of L points for many points, and the
// scratch bytes (meta, chunk offsets, partials with 16 B of alignment slack,
// segment sums and counts).
struct WalkLayout {
    int64_t target_chunks, max_chunks, L, blocks;
    int nb;
    bool multi;
    size_t bytes;
};

WalkLayout walk_layout(int64_t n, const Schedule &sc)
{
    constexpr int64_t kSegPoints = 2048, kMaxSegs = 1024;
    WalkLayout w{};
    w.target_chunks = (int64_t)device_cus() * 4 * 8 * sc.oversub;
    w.max_chunks = n + w.target_chunks + 1;
    w.multi = n > 8 * kSegPoints;
    w.nb = w.multi ? (int)std::min(kMaxSegs, (n + kSegPoints - 1) / kSegPoints) : 0;
    w.L = w.multi ? (n + w.nb - 1) / w.nb : 0;
    w.blocks = (w.max_chunks + kWalkBlock / kWave - 1) / (kWalkBlock / kWave);
    w.bytes = sizeof(int64_t) * (size_t)(n + 1) + 64 + 16 + sizeof(ChunkPartial) * (size_t)w.max_chunks +
              2 * sizeof(int64_t) * (size_t)w.nb;
    return w;
}

template <int KIND, int DATA, int PREC>
hipError_t run(const Geometry &g, const double *pts, int64_t n, const int64_t *walks, const int64_t *walk_begin,
               uint64_t seed, const uint64_t *node_seed, const uint32_t *stream_id, double *stats, int64_t *capped,
               const Schedule &sc, char *ws, hipStream_t s)
{
    const WalkLayout w = walk_layout(n, sc);
    const int64_t c_min = sc.min_chunk, target_chunks = w.target_chunks, max_chunks = w.max_chunks, L = w.L;
    const int nb = w.nb;
    if (w.blocks > 0x7fffffffLL) return hipErrorInvalidValue;
    hipError_t e;
    // scratch: the caller's workspace (at least w.bytes), else stream-ordered
    char *scratch = ws;
    if (!ws && (e = hipMallocAsync((void **)&scratch, w.bytes, s)) != hipSuccess) return e;
    int64_t *meta = (int64_t *)scratch;
    int64_t *chunk_off = (int64_t *)(scratch + 64);
    ChunkPartial *part = (ChunkPartial *)(scratch + 64 + sizeof(int64_t) * (size_t)(n + 1));
    if (((uintptr_t)part & 15u) != 0) part = (ChunkPartial *)(((uintptr_t)part + 15u) & ~(uintptr_t)15u);
    if (w.multi) {
        // segment sums and counts after the partials (the 16 spare bytes
        // cover the partials' alignment)
        int64_t *seg_part = (int64_t *)(part + max_chunks);
        int64_t *seg_cnt = seg_part + nb;
        hipLaunchKernelGGL(k_plan_sum, dim3(nb), dim3(kSegThreads), 0, s, walks, n, L, seg_part);
        hipLaunchKernelGGL(k_plan_count, dim3(nb), dim3(kSegThreads), 0, s, walks, n, L, seg_part, nb,
                           target_chunks, c_min, seg_cnt, meta);
        hipLaunchKernelGGL(k_plan_write, dim3(nb), dim3(kSegThreads), 0, s, walks, n, L, seg_cnt, chunk_off, meta);
    } else {
        hipLaunchKernelGGL(k_wos_plan, dim3(1), dim3(kPlanThreads), 0, s, walks, n, target_chunks, c_min, chunk_off,
                           meta);
    }
    hipLaunchKernelGGL((k_wos_walk<KIND, DATA, PREC>), dim3((unsigned)w.blocks), dim3(kWalkBlock), 0, s, g.dev, pts,
                       walks, walk_begin, stream_id, seed, node_seed, chunk_off, meta, n, part);
    hipLaunchKernelGGL((k_wos_finalize<KIND, DATA>), dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, g.dev, pts,
                       walks, n, chunk_off, part, stats, capped);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    return ws ? hipSuccess : hipFreeAsync(scratch, s);
}

template <int PREC>
hipError_t dispatch(const Geometry &g, const double *pts, int64_t n, const int64_t *walks, const int64_t *wb,
                    uint64_t seed, const uint64_t *ns, const uint32_t *sid, double *stats, int64_t *capped,
                    const Schedule &sc, char *ws, hipStream_t s)
{
    const bool src = g.dev.data_kind == DTN_DATA_POINT_SOURCES;
    constexpr int Q = DTN_DATA_HARMONIC_QUADRATIC, P = DTN_DATA_POINT_SOURCES;
    switch (g.dev.kind) {
    case DTN_BALL:
        return src ? run<DTN_BALL, P, PREC>(g, pts, n, walks, wb, seed, ns, sid, stats, capped, sc, ws, s)
                   : run<DTN_BALL, Q, PREC>(g, pts, n, walks, wb, seed, ns, sid, stats, capped, sc, ws, s);
    case DTN_BOX:
        if (g.dev.data_kind == DTN_DATA_TABULATED)
            return run<DTN_BOX, DTN_DATA_TABULATED, PREC>(g, pts, n, walks, wb, seed, ns, sid, stats, capped, sc, ws, s);
        return src ? run<DTN_BOX, P, PREC>(g, pts, n, walks, wb, seed, ns, sid, stats, capped, sc, ws, s)
                   : run<DTN_BOX, Q, PREC>(g, pts, n, walks, wb, seed, ns, sid, stats, capped, sc, ws, s);
    case DTN_HALF_SPACE:
        return src ? run<DTN_HALF_SPACE, P, PREC>(g, pts, n, walks, wb, seed, ns, sid, stats, capped, sc, ws, s)
                   : run<DTN_HALF_SPACE, Q, PREC>(g, pts, n, walks, wb, seed, ns, sid, stats, capped, sc, ws, s);
    case DTN_DISK:
        return src ? run<DTN_DISK, P, PREC>(g, pts, n, walks, wb, seed, ns, sid, stats, capped, sc, ws, s)
                   : run<DTN_DISK, Q, PREC>(g, pts, n, walks, wb, seed, ns, sid, stats, capped, sc, ws, s);
    case DTN_BALL_EXTERIOR:
        return src ? run<DTN_BALL_EXTERIOR, P, PREC>(g, pts, n, walks, wb, seed, ns, sid, stats, capped, sc, ws, s)
                   : run<DTN_BALL_EXTERIOR, Q, PREC>(g, pts, n, walks, wb, seed, ns, sid, stats, capped, sc, ws, s);
    default:
        if (!g.dev.cell_mask)
            return src ? run<kHolesNoGrid, P, PREC>(g, pts, n, walks, wb, seed, ns, sid, stats, capped, sc, ws, s)
                       : run<kHolesNoGrid, Q, PREC>(g, pts, n, walks, wb, seed, ns, sid, stats, capped, sc, ws, s);
        return src ? run<DTN_BOX_MINUS_BOXES, P, PREC>(g, pts, n, walks, wb, seed, ns, sid, stats, capped, sc, ws, s)
                   : run<DTN_BOX_MINUS_BOXES, Q, PREC>(g, pts, n, walks, wb, seed, ns, sid, stats, capped, sc, ws, s);
    }
}

hipError_t walk_all(const Geometry &g, const double *pts, int64_t n, const int64_t *walks, const int64_t *walk_begin,
                    uint64_t seed, const uint64_t *node_seed, const uint32_t *stream_id, int precision,
                    double *stats, int64_t *capped, const Schedule &sc, hipStream_t stream, char *ws = nullptr)
{
    return precision == DTN_FP64
               ? dispatch<DTN_FP64>(g, pts, n, walks, walk_begin, seed, node_seed, stream_id, stats, capped, sc, ws,
                                    stream)
               : dispatch<DTN_FP32_MIXED>(g, pts, n, walks, walk_begin, seed, node_seed, stream_id, stats, capped,
                                          sc, ws, stream);
}

// ------------------------------------------------- distance (diagnostic)

template <int KIND, bool FAST>
__global__ __launch_bounds__(256) void k_distance(DevGeom g, const double *__restrict__ pts, int64_t n,
                                                  double *__restrict__ out)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const bool live = i < n;
    const double x = live ? pts[3 * i] : 0.0, y = live ? pts[3 * i + 1] : 0.0, z = live ? pts[3 * i + 2] : 0.0;
    uint32_t cand = 0;
    if constexpr (KIND == DTN_BOX_MINUS_BOXES) cand = hole_candidates(g, cell_offsets(g), live, (float)x, (float)y, (float)z);
    if (!live) return;
    out[i] = dist_f64<KIND, FAST>(g, x, y, z, cand);
}

template <bool FAST>
void distance_kind(const Geometry &g, const double *pts, int64_t n, double *out, hipStream_t s)
{
    const dim3 grid((unsigned)((n + 255) / 256)), block(256);
    switch (g.dev.kind) {
    case DTN_BALL: hipLaunchKernelGGL((k_distance<DTN_BALL, FAST>), grid, block, 0, s, g.dev, pts, n, out); break;
    case DTN_BOX: hipLaunchKernelGGL((k_distance<DTN_BOX, FAST>), grid, block, 0, s, g.dev, pts, n, out); break;
    case DTN_HALF_SPACE:
        hipLaunchKernelGGL((k_distance<DTN_HALF_SPACE, FAST>), grid, block, 0, s, g.dev, pts, n, out);
        break;
    case DTN_DISK: hipLaunchKernelGGL((k_distance<DTN_DISK, FAST>), grid, block, 0, s, g.dev, pts, n, out); break;
    case DTN_BALL_EXTERIOR:
        hipLaunchKernelGGL((k_distance<DTN_BALL_EXTERIOR, FAST>), grid, block, 0, s, g.dev, pts, n, out);
        break;
    default:
        if (g.dev.cell_mask)
            hipLaunchKernelGGL((k_distance<DTN_BOX_MINUS_BOXES, FAST>), grid, block, 0, s, g.dev, pts, n, out);
        else
            hipLaunchKernelGGL((k_distance<kHolesNoGrid, FAST>), grid, block, 0, s, g.dev, pts, n, out);
    }
}

// ------------------------------------------------------- adaptive budgets

__global__ __launch_bounds__(256) void k_fill_i64(int64_t *__restrict__ a, int64_t n, int64_t v)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) a[i] = v;
}

// Per point: total walks = clamp(ceil(var / se^2), w_min, w_max), never fewer
// than the pilot; the remainder continues at walk index `pilot`.
__global__ __launch_bounds__(256) void k_budget(const double *__restrict__ pilot_stats, int64_t n, int64_t pilot,
                                                int64_t w_min, int64_t w_max, double se2_all,
                                                const double *__restrict__ node_se2,
                                                int64_t *__restrict__ rem, int64_t *__restrict__ wb,
                                                int64_t *__restrict__ used)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const double se2 = node_se2 ? node_se2[i] : se2_all;
    const double cnt = pilot_stats[4 * i], m2 = pilot_stats[4 * i + 2];
    const double var = cnt > 1.0 ? m2 / (cnt - 1.0) : 0.0;
    const double want = ceil(var / se2);
    int64_t tot;
    if (!(want < (double)w_max)) tot = w_max;  // also catches NaN
    else if (want <= (double)w_min) tot = w_min;
    else tot = (int64_t)want;
    tot = max(tot, pilot);
    rem[i] = tot - pilot;
    wb[i] = pilot;
    used[i] = tot;
}

// Merge the pilot statistics with the remainder's (Chan, Golub & LeVeque's
// pairwise update of count, mean and sum of squared deviations).
__global__ __launch_bounds__(256) void k_merge(const double *__restrict__ ps, const int64_t *__restrict__ pcap,
                                               const int64_t *__restrict__ rcap, double *__restrict__ stats,
                                               int64_t *__restrict__ capped, int64_t n)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const double n1 = ps[4 * i], m1 = ps[4 * i + 1], M1 = ps[4 * i + 2], t1 = ps[4 * i + 3];
    const double n2 = stats[4 * i], m2 = stats[4 * i + 1], M2 = stats[4 * i + 2], t2 = stats[4 * i + 3];
    double cnt = n1, mean = m1, msq = M1;
    if (n2 > 0.0) {
        cnt = n1 + n2;
        const double d = m2 - m1;
        mean = m1 + d * (n2 / cnt);
        msq = M1 + M2 + d * d * (n1 * (n2 / cnt));
    }
    stats[4 * i] = cnt;
    stats[4 * i + 1] = mean;
    stats[4 * i + 2] = msq;
    stats[4 * i + 3] = t1 + t2;
    if (capped) capped[i] = pcap[i] + rcap[i];
}

}  // namespace

// Status of a geometry: snapshot the live bits (or the walk counters) and
// clear them in one atomic exchange each (work still running on other
// streams keeps raising them).
__global__ void k_take_status(DevStatus *st, int counters)
{
    if (threadIdx.x != 0) return;
    if (counters) {
        st->iters_taken = atomicExch(&st->iters, 0ull);
        st->visits_taken = atomicExch(&st->visits, 0ull);
    } else {
        st->flags_taken = atomicExch(&st->flags, 0u);
    }
}

dtn_status take_flags(const Geometry &g, hipStream_t s, uint32_t &out)
{
    out = 0;
    hipLaunchKernelGGL(k_take_status, dim3(1), dim3(kWave), 0, s, g.d_status, 0);
    hipError_t e = hipGetLastError();
    if (e == hipSuccess)
        e = hipMemcpyAsync(&out, &g.d_status->flags_taken, sizeof(uint32_t), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return fail(DTN_E_DEVICE, std::string("dtn_check: ") + hipGetErrorString(e));
    return DTN_OK;
}

dtn_status take_counters(const Geometry &g, hipStream_t s, unsigned long long out[2])
{
    out[0] = out[1] = 0;
    hipLaunchKernelGGL(k_take_status, dim3(1), dim3(kWave), 0, s, g.d_status, 1);
    hipError_t e = hipGetLastError();
    if (e == hipSuccess)
        e = hipMemcpyAsync(out, &g.d_status->iters_taken, 2 * sizeof(unsigned long long), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return fail(DTN_E_DEVICE, std::string("dtn_walk_counters: ") + hipGetErrorString(e));
    return DTN_OK;
}

dtn_status launch_wos(const Geometry &g, const double *pts, int64_t n, const int64_t *walks,
                      const int64_t *walk_begin, uint64_t seed, const uint32_t *stream_id, int precision,
                      double *stats, int64_t *capped, const Schedule &sc, hipStream_t stream)
{
    if (n == 0) return DTN_OK;
    hipError_t e =
        walk_all(g, pts, n, walks, walk_begin, seed, nullptr, stream_id, precision, stats, capped, sc, stream);
    if (e != hipSuccess) return fail(DTN_E_DEVICE, std::string("dtn_wos_eval: ") + hipGetErrorString(e));
    return DTN_OK;
}

// Workspace of the walk launches of dtn_wos_eval_noalloc: one copy per
// device, held until the process ends.  Host code never passes the array's
// name to a kernel (on the host it is a stand-in, not a device address): it
// takes the device's address once, with that device current, and passes
// that.  Nothing in it needs clearing: every word a launch reads (chunk
// offsets, meta, partials, segment sums) is written earlier in the same
// launch sequence.
constexpr size_t kNoAllocBytes = (size_t)64 << 20;
static __device__ __align__(256) char scratch[kNoAllocBytes];

namespace {

std::mutex g_scratch_mu;
std::map<int, char *> g_scratch_ptr;  // device -> address of its `scratch`

dtn_status device_scratch(char **out)
{
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return fail(DTN_E_DEVICE, std::string("dtn_wos_eval_noalloc: ") + hipGetErrorString(e));
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    auto it = g_scratch_ptr.find(dev);
    if (it == g_scratch_ptr.end()) {
        void *ptr = nullptr;
        e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !ptr)
            return fail(DTN_E_DEVICE, std::string("dtn_wos_eval_noalloc: workspace address: ") +
                                          hipGetErrorString(e));
        it = g_scratch_ptr.emplace(dev, (char *)ptr).first;
    }
    *out = it->second;
    return DTN_OK;
}

}  // namespace

size_t noalloc_workspace_bytes() { return kNoAllocBytes; }
size_t noalloc_bytes(int64_t n) { return walk_layout(n, Schedule{}).bytes; }

dtn_status launch_wos_noalloc(const Geometry &g, const double *pts, int64_t n, const int64_t *walks,
                              const int64_t *walk_begin, uint64_t seed, const uint32_t *stream_id, int precision,
                              double *stats, int64_t *capped, hipStream_t stream)
{
    if (n == 0) return DTN_OK;
    const Schedule sc;
    const size_t need = walk_layout(n, sc).bytes;
    if (need > kNoAllocBytes)
        return fail(DTN_E_ARG, "dtn_wos_eval_noalloc: " + std::to_string(n) + " points need " + std::to_string(need) +
                                   " bytes of workspace, more than its " + std::to_string(kNoAllocBytes));
    char *ptr = nullptr;
    const dtn_status st = device_scratch(&ptr);
    if (st != DTN_OK) return st;
    const hipError_t e =
        walk_all(g, pts, n, walks, walk_begin, seed, nullptr, stream_id, precision, stats, capped, sc, stream, ptr);
    if (e != hipSuccess) return fail(DTN_E_DEVICE, std::string("dtn_wos_eval_noalloc: ") + hipGetErrorString(e));
    return DTN_OK;
}

dtn_status launch_distance(const Geometry &g, const double *pts, int64_t n, int precision, double *dist,
                           hipStream_t stream)
{
    if (n == 0) return DTN_OK;
    if (precision == DTN_FP64) distance_kind<false>(g, pts, n, dist, stream);
    else distance_kind<true>(g, pts, n, dist, stream);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return fail(DTN_E_DEVICE, std::string("dtn_boundary_distance: ") + hipGetErrorString(e));
    return DTN_OK;
}

dtn_status launch_wos_adaptive(const Geometry &g, const double *pts, int64_t n, const Adaptive &a, uint64_t seed,
                               const uint64_t *node_seed,
                               const uint32_t *stream_id, int precision, double *stats, int64_t *walks_used,
                               int64_t *capped, const Schedule &sc, hipStream_t s)
{
    if (n == 0) return DTN_OK;
    const char *where = "dtn_wos_adaptive: ";
    // scratch: pilot stats [n][4] doubles, then pilot walks, remainder walks,
    // remainder first walk, pilot capped, remainder capped ([n] int64 each)
    char *scratch = nullptr;
    const size_t bytes = (size_t)n * (4 * sizeof(double) + 5 * sizeof(int64_t));
    hipError_t e = hipMallocAsync((void **)&scratch, bytes, s);
    if (e != hipSuccess) return fail(DTN_E_OOM, std::string(where) + hipGetErrorString(e));
    double *pstats = (double *)scratch;
    int64_t *pw = (int64_t *)(scratch + (size_t)n * 4 * sizeof(double));
    int64_t *rw = pw + n, *wb = rw + n, *pcap = wb + n, *rcap = pcap + n;
    const unsigned grid = (unsigned)((n + 255) / 256);
    hipLaunchKernelGGL(k_fill_i64, dim3(grid), dim3(256), 0, s, pw, n, a.pilot);
    e = walk_all(g, pts, n, pw, nullptr, seed, node_seed, stream_id, precision, pstats, pcap, sc, s);
    if (e == hipSuccess) {
        hipLaunchKernelGGL(k_budget, dim3(grid), dim3(256), 0, s, pstats, n, a.pilot, a.w_min, a.w_max,
                           a.se * a.se, a.node_se2, rw, wb, walks_used);
        e = walk_all(g, pts, n, rw, wb, seed, node_seed, stream_id, precision, stats, rcap, sc, s);
    }
    if (e == hipSuccess) {
        hipLaunchKernelGGL(k_merge, dim3(grid), dim3(256), 0, s, pstats, pcap, rcap, stats, capped, n);
        e = hipGetLastError();
    }
    const hipError_t ef = hipFreeAsync(scratch, s);
    if (e == hipSuccess) e = ef;
    if (e != hipSuccess) return fail(DTN_E_DEVICE, std::string(where) + hipGetErrorString(e));
    return DTN_OK;
}

}  // namespace dtn
