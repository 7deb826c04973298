// Single-wave and whole-workgroup helpers of the small FP64 algebra: LDS
// matrix moves and products, fixed-order sums of per-workgroup partials, a
// two-at-once Cholesky factorisation with inverses, and a one-sided Jacobi
// SVD run by one wave. Shared by the panel kernels of the loop and of the
// relaxed iteration.
#pragma once

#include "launch.hpp"

namespace rpca {
namespace {

constexpr double JACOBI_EPS = 1e-15;
// Pairs with |a_p . a_q| <= JACOBI_ABS ||M||_F^2 are left alone: such a coupling
// moves the leading singular vectors by about that relative amount, and the
// trailing (negligible) columns would otherwise keep rotating on rounding noise.
constexpr double JACOBI_ABS = 1e-17;
constexpr int JACOBI_MAX_SWEEPS = 40;
// Cyclic Jacobi converges quadratically: once every rotation of a sweep was by
// an angle below JACOBI_QUAD (the angle is the coupling over the gap of the
// pair), the angles a further sweep would take are of the order
// JACOBI_QUAD^2, and the confirming sweep is skipped.
constexpr double JACOBI_QUAD = 1e-8;
// The same for M formed from FP32 products: the angles a further sweep would
// take (about 4e-8) are below the rounding of those products (6e-8) and of the
// FP32 factors the result is stored in, and below the initial subspace
// iteration's FP32 tolerance (3e-6), so stopping here changes nothing the FP32
// path can resolve. It saves about one sweep of the single-wave tail per body.
constexpr double JACOBI_QUAD_F32 = 2e-4;
constexpr double CHOL_DEAD_REL = 1e-26;

// ---- single-wave helpers (the last workgroup's tail) ---------------------------

__device__ inline int lane_id() { return threadIdx.x & (WAVE - 1); }
__device__ inline void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
}

template <int K>
__device__ inline void w_load(const double* __restrict__ g, double* s) {
    for (int e = lane_id(); e < K * K; e += WAVE) s[e] = g[(e / K) * KMAX + (e % K)];
    wave_sync();
}
template <int K>
__device__ inline void w_store(const double* s, double* __restrict__ g) {
    for (int e = lane_id(); e < K * K; e += WAVE) g[(e / K) * KMAX + (e % K)] = s[e];
    wave_sync();
}
// Global -> registers -> LDS in two steps, so that the load can be issued
// early and its latency overlap other work: lane l holds entries l, l + WAVE, ...
template <int K> constexpr int w_per_lane() { return (K * K + WAVE - 1) / WAVE; }
template <int K>
__device__ inline void w_fetch(const double* __restrict__ g, double (&v)[w_per_lane<K>()]) {
#pragma unroll
    for (int u = 0; u < w_per_lane<K>(); ++u) {
        const int e = lane_id() + u * WAVE;
        v[u] = e < K * K ? g[(e / K) * KMAX + (e % K)] : 0.0;
    }
}
template <int K>
__device__ inline void w_put(const double (&v)[w_per_lane<K>()], double* s) {
#pragma unroll
    for (int u = 0; u < w_per_lane<K>(); ++u) {
        const int e = lane_id() + u * WAVE;
        if (e < K * K) s[e] = v[u];
    }
    wave_sync();
}
// C = op(A) B (K x K, ld K, LDS); op = transpose when TA
template <int K, bool TA>
__device__ inline void w_mm(const double* A, const double* B, double* C) {
    for (int e = lane_id(); e < K * K; e += WAVE) {
        const int i = e / K, j = e % K;
        double acc = 0.0;
        for (int l = 0; l < K; ++l) acc = fma(TA ? A[l * K + i] : A[i * K + l], B[l * K + j], acc);
        C[e] = acc;
    }
    wave_sync();
}
// Two independent products C = op(A) B and F = op(D) E in one pass
template <int K, bool TA>
__device__ inline void w_mm2(const double* A, const double* B, double* C, const double* D, const double* E,
                             double* F) {
    for (int x = lane_id(); x < 2 * K * K; x += WAVE) {
        const bool second = x >= K * K;
        const int e = second ? x - K * K : x;
        const double* P = second ? D : A;
        const double* Q = second ? E : B;
        const int i = e / K, j = e % K;
        double acc = 0.0;
        for (int l = 0; l < K; ++l) acc = fma(TA ? P[l * K + i] : P[i * K + l], Q[l * K + j], acc);
        (second ? F : C)[e] = acc;
    }
    wave_sync();
}

// Sums of the per-workgroup partials of a kernel whose first gU workgroups
// cover the U side (rows of m) and the next gV the V side (rows of n). Job j
// sums entry e < E of the partial at offset (j / 2) * KMAX^2 of every
// workgroup of side j % 2, into out[j * E + e].
// The whole workgroup (NT threads) takes part. Thread t takes pair
// q = t % PAIRS (job q / E, entry q % E) and split s = t / PAIRS and sums the
// partials b = s, s + S, ... in order; the S split sums of a pair are then
// added in order of s. Up to L loads per thread are in flight at once, so a
// round over up to L S partials costs one memory latency. part: NT doubles
// of LDS.
template <int E, int J, int NT, int L = 16>
__device__ __forceinline__ void block_sum_partials(const double* __restrict__ gpart, int gU, int gV, double* out, double* part) {
    constexpr int PAIRS = J * E;
    constexpr int PR = PAIRS >= NT ? NT : PAIRS;   // pairs per round
    constexpr int S = NT / PR;                     // splits per pair
    // L: loads in flight per thread
    const int t = threadIdx.x;
    for (int q0 = 0; q0 < PAIRS; q0 += PR) {
        const int sp = t / PR, q = q0 + t % PR;
        double acc = 0.0;
        if (sp < S && q < PAIRS) {
            const int j = q / E, e = q - (q / E) * E;
            const int first = (j & 1) ? gU : 0, count = (j & 1) ? gV : gU;
            const double* g = gpart + (size_t)first * GPART_STRIDE + (j >> 1) * (KMAX * KMAX) + e;
            for (int b0 = sp; b0 < count; b0 += L * S) {
                double v[L];
#pragma unroll
                for (int u = 0; u < L; ++u) {
                    const int b = b0 + u * S;
                    v[u] = b < count ? g[(size_t)b * GPART_STRIDE] : 0.0;
                }
#pragma unroll
                for (int u = 0; u < L; ++u) acc += v[u];
            }
        }
        if (t < S * PR) part[t] = acc;
        __syncthreads();
        if (t < PR && q0 + t < PAIRS) {
            double v = 0.0;
            for (int u = 0; u < S; ++u) v += part[u * PR + t];
            out[q0 + t] = v;
        }
        __syncthreads();
    }
}

template <int CTRL> __device__ inline double dpp64(double x);
__device__ inline double row16_sum(double x);
__device__ inline double row16_max(double x);
__device__ inline double readlane64(double x, int l);

// Sum of the per-tile residuals (and, if want_max, the max of the per-tile
// max |D_ij| stored after them) by the whole workgroup, in a fixed order.
// out[0] = sum, out[1] = max. part: at least 2 * NT / 16 doubles of LDS.
// Split in two: block_resid_fetch issues the loads of the first RESID_LD * NT
// tiles into registers (so that other loads can follow before they are
// used), block_resid adds them, and any further tiles, in tile order per thread.
constexpr int RESID_LD = 2;
template <int NT>
__device__ inline void block_resid_fetch(const double* __restrict__ resid, int n_tiles, bool want_max,
                                         double (&v)[RESID_LD], double (&w)[RESID_LD]) {
#pragma unroll
    for (int u = 0; u < RESID_LD; ++u) {
        const int b = threadIdx.x + u * NT;
        v[u] = b < n_tiles ? resid[b] : 0.0;
        w[u] = (want_max && b < n_tiles) ? resid[n_tiles + b] : 0.0;
    }
}
template <int NT>
__device__ __forceinline__ void block_resid(const double* __restrict__ resid, int n_tiles, bool want_max,
                            const double (&v)[RESID_LD], const double (&w)[RESID_LD], double* part, double* out) {
    const int t = threadIdx.x;
    double sm = 0.0, mx = 0.0;
#pragma unroll
    for (int u = 0; u < RESID_LD; ++u) {
        sm += v[u];
        mx = fmax(mx, w[u]);
    }
    for (int b = t + RESID_LD * NT; b < n_tiles; b += NT) {
        sm += resid[b];
        if (want_max) mx = fmax(mx, resid[n_tiles + b]);
    }
    // sums and maxima over each row of 16 lanes by DPP; the four rows of a
    // wave go to LDS separately
    sm = row16_sum(sm);
    mx = row16_max(mx);
    constexpr int NW = NT / 16;
    static_assert(NW <= WAVE, "one row sum per lane of the first wave");
    if ((t & 15) == 0) {
        part[t / 16] = sm;
        part[NW + t / 16] = mx;
    }
    __syncthreads();
    if (t < WAVE) {
        double a = t < NW ? part[t] : 0.0, m = t < NW ? part[NW + t] : 0.0;
        a = row16_sum(a);
        m = row16_max(m);
        a = (readlane64(a, 0) + readlane64(a, 16)) + (readlane64(a, 32) + readlane64(a, 48));
        m = fmax(fmax(readlane64(m, 0), readlane64(m, 16)), fmax(readlane64(m, 32), readlane64(m, 48)));
        if (t == 0) {
            out[0] = a;
            out[1] = m;
        }
    }
    __syncthreads();
}

__device__ inline double readlane64(double x, int l) {
    const int64_t u = __double_as_longlong(x);
    const int lo = __builtin_amdgcn_readlane((int)(uint32_t)u, l);
    const int hi = __builtin_amdgcn_readlane((int)(uint32_t)(u >> 32), l);
    return __longlong_as_double((int64_t)(((uint64_t)(uint32_t)hi << 32) | (uint32_t)lo));
}

// Two Cholesky factorisations at once, G0 = R0^T R0 in lanes 0..31 and
// G1 = R1^T R1 in lanes 32..63, with the inverses R^{-1} (all K x K, ld K,
// LDS; R upper triangular). Lane c of a half owns column c in registers; the
// factorisation is right-looking: at step j the pivot and row j of R are
// formed in registers and broadcast with readlane, and the trailing columns
// are updated. A pivot that vanishes (d <= CHOL_DEAD_REL * G_jj, or G_jj ~ 0)
// marks a numerically dependent column: its row of R and column of R^{-1}
// are 0. R^{-1} by back substitution from R in LDS, column c in lane c.
template <int K>
__device__ __forceinline__ void w_chol_inv2(const double* G0, double* R0, double* Ri0, const double* G1, double* R1,
                            double* Ri1) {
    static_assert(K <= 32, "one column per lane of a half wave");
    const int lane = lane_id();
    const int h = lane >> 5, c = lane & 31;
    const double* G = h ? G1 : G0;
    double g[K], r[K], inv[K], x[K];
#pragma unroll
    for (int i = 0; i < K; ++i) g[i] = c < K ? G[i * K + c] : 0.0;
#pragma unroll
    for (int j = 0; j < K; ++j) {
        const double d = h ? readlane64(g[j], 32 + j) : readlane64(g[j], j);
        const double gjj = G[j * K + j];
        const bool live = gjj > 1e-300 && d > CHOL_DEAD_REL * gjj;
        const double ivj = live ? rsqrt(d) : 0.0;   // one reciprocal square root, no division
        const double rjj = live ? d * ivj : 0.0;
        inv[j] = ivj;
        r[j] = (c == j) ? rjj : (c > j ? g[j] * ivj : 0.0);   // R[j][c]
#pragma unroll
        for (int i = j + 1; i < K; ++i) {
            const double rji = h ? readlane64(r[j], 32 + i) : readlane64(r[j], i);
            g[i] = fma(-rji, r[j], g[i]);
        }
    }
    double* R = h ? R1 : R0;
    double* Ri = h ? Ri1 : Ri0;
    if (c < K) {
#pragma unroll
        for (int i = 0; i < K; ++i) R[i * K + c] = r[i];
    }
    wave_sync();
    // back substitution with R read from LDS (same address in all lanes of a half)
#pragma unroll
    for (int i = K - 1; i >= 0; --i) {
        double v = (i == c) ? 1.0 : 0.0;
#pragma unroll
        for (int k = i + 1; k < K; ++k) v = fma(-R[i * K + k], x[k], v);
        x[i] = v * inv[i];
    }
    if (c < K) {
#pragma unroll
        for (int i = 0; i < K; ++i) Ri[i * K + c] = x[i];
    }
    wave_sync();
}

template <int CTRL> __device__ inline double dpp64(double x) {
    const int64_t u = __double_as_longlong(x);
    const int lo = __builtin_amdgcn_update_dpp(0, (int)(uint32_t)u, CTRL, 0xf, 0xf, true);
    const int hi = __builtin_amdgcn_update_dpp(0, (int)(uint32_t)(u >> 32), CTRL, 0xf, 0xf, true);
    return __longlong_as_double((int64_t)(((uint64_t)(uint32_t)hi << 32) | (uint32_t)lo));
}
__device__ inline double row16_sum(double x) {
    x += dpp64<0xB1>(x);
    x += dpp64<0x4E>(x);
    x += dpp64<0x141>(x);
    x += dpp64<0x128>(x);
    return x;
}
__device__ inline double row16_max(double x) {
    x = fmax(x, dpp64<0xB1>(x));
    x = fmax(x, dpp64<0x4E>(x));
    x = fmax(x, dpp64<0x141>(x));
    x = fmax(x, dpp64<0x128>(x));
    return x;
}
// Sum over aligned groups of LP lanes (LP = 1, 2, 4, 8, 16), result in every lane.
template <int LP> __device__ inline double group_sum(double x) {
    if constexpr (LP >= 2) x += dpp64<0xB1>(x);    // quad_perm[1,0,3,2]: lane ^ 1
    if constexpr (LP >= 4) x += dpp64<0x4E>(x);    // quad_perm[2,3,0,1]: lane ^ 2
    if constexpr (LP >= 8) x += dpp64<0x141>(x);   // row_half_mirror:    lane ^ 7
    if constexpr (LP >= 16) x += dpp64<0x128>(x);  // row_ror:8:          lane ^ 8
    return x;
}

constexpr int pow2_floor(int x) { int p = 1; while (p * 2 <= x) p *= 2; return p; }

// One-sided (Hestenes) Jacobi SVD of the N x N matrix A (LDS, column-major),
// run by a single wave: the N/2 disjoint column pairs of a round-robin round
// are processed at once, LP lanes per pair, with DPP reductions for the three
// inner products. A pair is rotated when |a_p . a_q| > JACOBI_EPS ||a_p|| ||a_q||
// and above the absolute floor JACOBI_ABS ||A||_F^2 (pairs of negligible
// columns would otherwise rotate on rounding noise), unless both columns have
// ||a||^2 <= neg2 ||A||_F^2 (columns the caller discards: a rotation never
// raises the smaller norm of a pair). Sweeps stop when no pair was rotated, or
// (QUAD_STOP) after a sweep whose rotation angles were all below
// quad (default JACOBI_QUAD); callers that difference the result keep the
// confirming sweep. On return
// sig[] is descending and Uo/Vo hold the left/right singular vectors as
// columns (column-major). Returns the sweep count.
template <int N, bool QUAD_STOP = true>
__device__ __forceinline__ int wave_jacobi_svd(double* A, double* V, double* sig, double* Uo, double* Vo, double neg2 = 0.0,
                                               double quad = JACOBI_QUAD) {
    static_assert(N % 2 == 0 && N <= 2 * KMAX, "even N up to 2*KMAX");
    constexpr int NP = N / 2;
    constexpr int LP0 = pow2_floor(WAVE / NP);
    constexpr int LP = LP0 > 16 ? 16 : LP0;
    constexpr int E = (N + LP - 1) / LP;
    const int lane = lane_id();
    double fro = 0.0;
    for (int e = lane; e < N * N; e += WAVE) {
        V[e] = ((e / N) == (e % N)) ? 1.0 : 0.0;
        fro = fma(A[e], A[e], fro);
    }
    for (int off = 32; off > 0; off >>= 1) fro += __shfl_xor(fro, off, WAVE);
    const double floor_abs = JACOBI_ABS * fro;
    const double floor_neg = neg2 * fro;
    wave_sync();
    const int q = lane / LP, g = lane % LP;
    int sweep = 0;
    for (; sweep < JACOBI_MAX_SWEEPS; ++sweep) {
        bool rotated = false, large = false;
        for (int rd = 0; rd < N - 1; ++rd) {
            if (q < NP) {
                const int a = (q == 0) ? 0 : ((q - 1 + rd) % (N - 1)) + 1;
                const int b = ((N - 2 - q + rd) % (N - 1)) + 1;
                double xa[E], xb[E], va[E], vb[E];
                double al = 0.0, be = 0.0, ga = 0.0;
#pragma unroll
                for (int u = 0; u < E; ++u) {
                    const int e = g + LP * u;
                    const bool ok = e < N;
                    xa[u] = ok ? A[a * N + e] : 0.0;
                    xb[u] = ok ? A[b * N + e] : 0.0;
                    va[u] = ok ? V[a * N + e] : 0.0;
                    vb[u] = ok ? V[b * N + e] : 0.0;
                    al = fma(xa[u], xa[u], al);
                    be = fma(xb[u], xb[u], be);
                    ga = fma(xa[u], xb[u], ga);
                }
                al = group_sum<LP>(al);
                be = group_sum<LP>(be);
                ga = group_sum<LP>(ga);
                if (ga * ga > (JACOBI_EPS * JACOBI_EPS) * (al * be) && fabs(ga) > floor_abs &&
                    fmax(al, be) > floor_neg) {

                    // rotation by theta, |theta| <= pi/4, tan 2 theta = 2 ga / (be - al):
                    // with h = sqrt((be - al)^2 + 4 ga^2), cos 2 theta = |be - al| / h,
                    // c = sqrt((1 + cos 2 theta) / 2), s = sign(be - al) ga / (h c);
                    // two reciprocal square roots, no division
                    const double dl = be - al;
                    const double rh = rsqrt(fma(dl, dl, 4.0 * ga * ga));
                    const double c2 = fma(0.5 * fabs(dl), rh, 0.5);
                    const double ic = rsqrt(c2);
                    const double c = c2 * ic;
                    const double s = (dl >= 0.0 ? ga : -ga) * rh * ic;
                    large = large || fabs(s) > quad;
#pragma unroll
                    for (int u = 0; u < E; ++u) {
                        const int e = g + LP * u;
                        if (e < N) {
                            A[a * N + e] = c * xa[u] - s * xb[u];
                            A[b * N + e] = s * xa[u] + c * xb[u];
                            V[a * N + e] = c * va[u] - s * vb[u];
                            V[b * N + e] = s * va[u] + c * vb[u];
                        }
                    }
                    rotated = true;
                }
            }
            wave_sync();
        }
        if (!__any(rotated)) break;
        if (QUAD_STOP && !__any(large)) { ++sweep; break; }
    }
    // column norms, ranks (descending, ties by index), normalised outputs
    if (lane < N) {
        double acc = 0.0;
        for (int e = 0; e < N; ++e) acc = fma(A[lane * N + e], A[lane * N + e], acc);
        sig[lane] = sqrt(acc);
    }
    wave_sync();
    double sj = 0.0;
    int rank = 0;
    if (lane < N) {
        sj = sig[lane];
        for (int i = 0; i < N; ++i) {
            const double si = sig[i];
            rank += (si > sj) || (si == sj && i < lane);
        }
    }
    wave_sync();
    if (lane < N) {
        sig[rank] = sj;
        const double inv = sj > 0.0 ? 1.0 / sj : 0.0;
        for (int e = 0; e < N; ++e) {
            Uo[rank * N + e] = A[lane * N + e] * inv;
            Vo[rank * N + e] = V[lane * N + e];
        }
    }
    wave_sync();
    return sweep + 1;
}

// ---- the update kernel's closing sums -----------------------------------------
//
// Sums of the per-workgroup partials the update kernel leaves in gpart (gU U
// side, gV V side) and what follows from them: Gram(U_f) = R_U^T R_U and
// Gram(V_f) = R_V^T R_V (R^{-1} by Cholesky, into RUinv/RVinv, or RAinv/RBinv
// for the exact bases) and, with cross, A_L^T U_f and B_L^T V_f (GAU, GBV)
// for the gather of the next rebuilding pass. The whole workgroup (NT threads)
// sums in a fixed order; its first wave factorises. Run by the update kernel's
// last workgroup when it enters from a given state, and otherwise by the first
// workgroup to finish the streaming pass that follows (ctrl->post_update).
// L: loads in flight per thread (the order of the sums, and so the result,
// does not depend on it). lds: FINISH_LDS<K, NT>() doubles of LDS scratch.
template <int K, int NT> constexpr int FINISH_LDS() { return 8 * K * K + NT; }
template <int K, int NT, int L>
__device__ __forceinline__ void finish_basis(const double* __restrict__ gpart, int gU, int gV, bool cross,
                                             bool exact, Small* sm, double* lds) {
    double* gg = lds;                 // 4 K^2: the four sums
    double* rr = gg + 4 * K * K;      // K^2 each: R_U, R_U^{-1}, R_V, R_V^{-1}
    double* ri = rr + K * K;
    double* rr2 = ri + K * K;
    double* ri2 = rr2 + K * K;
    double* part = ri2 + K * K;       // NT
    if (cross) block_sum_partials<K * K, 4, NT, L>(gpart, gU, gV, gg, part);
    else block_sum_partials<K * K, 2, NT, L>(gpart, gU, gV, gg, part);
    if (threadIdx.x < WAVE) {
        if (cross) {
            w_store<K>(gg + 2 * K * K, sm->GAU);
            w_store<K>(gg + 3 * K * K, sm->GBV);
        }
        w_chol_inv2<K>(gg, rr, ri, gg + K * K, rr2, ri2);
        w_store<K>(ri, exact ? sm->RAinv : sm->RUinv);
        w_store<K>(ri2, exact ? sm->RBinv : sm->RVinv);
    }
}

// End of a streaming-pass workgroup: workgroup 0 of the launch (of each
// instance), which starts first on its CU and is among the first to finish,
// completes the update kernel that preceded the pass when that kernel left
// its closing sums to the pass (post_update 1: Grams, 2: Grams and cross
// products). Its results are first read by the gather after the pass. The
// flag is set by the update kernel and cleared here and by every other kernel
// that overwrites the partials.
// lds: FINISH_LDS<K, NT>() doubles of the pass's LDS, free once its tile is
// done (the barrier below separates the two uses).
template <int K, int NT>
__device__ __forceinline__ void pass_finishes_update(Ctrl* ctrl, const StreamGeom& g, int64_t off, double* lds) {
    if (g.post_gpart == nullptr || blockIdx.x != 0) return;
    const int mode = ctrl->post_update;
    if (mode == 0) return;
    __syncthreads();
    // 32 loads in flight per thread, as in the update kernel: with fewer, a
    // sum over the 2 x 79 partials of m = n = 2 10^4 takes tens of dependent
    // round trips and can outlast the pass (the pass's own registers still
    // bound the kernel's)
    finish_basis<K, NT, 32>(moved(g.post_gpart, off), g.post_gU, g.post_gV, mode == 2, false,
                           moved(g.post_small, off), lds);
    if (threadIdx.x == 0) ctrl->post_update = 0;
}

}  // namespace
}  // namespace rpca
