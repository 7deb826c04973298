// Tall-skinny (m x K, n x K) FP64 panel kernels between two streaming passes,
// and the small K x K / 2K x 2K FP64 linear algebra of Section 2.1.
//
// Every panel kernel runs one thread per row over the m rows of the U side and
// the n rows of the V side in one grid. Reductions over rows (Gram matrices,
// U_f^T Y1) are written as per-workgroup partials; the workgroup that
// finishes last (atomic arrival counter + device-scope fences) sums them in a
// fixed order and runs the small dense algebra, so results are deterministic.
//
// Notation (k-th iteration, K = r in the loop and K = p in the initialisation):
//   U_f, V_f   bases used by the streaming pass (dtype of D)
//   R_U, R_V   Cholesky factors of Gram(U_f), Gram(V_f); U* = U_f R_U^{-1} and
//              V* = V_f R_V^{-1} are orthonormal to FP64 accuracy and span the
//              same spaces, so the FP32 rounding of the bases never breaks the
//              orthogonality the 2r x 2r reduction relies on
//   Y1 = Z V_f, Y2 = Z^T U_f                (streaming pass, Z = D - S_k)
//   C*  = U*^T Z V*                         top-left block of M
//   W1  = (I - U* U*^T) Z V* = Q1 R1,  W2 = (I - V* V*^T) Z^T U* = Q2 R2
//   M   = [[C*, R2^T], [R1, 0]] = U_M Sigma_M V_M^T   (one-sided Jacobi)
//   U_{k+1} = [U* Q1] U_M[:, :K] = U* X1 + W1 X2,  X2 = R1^{-1} U_M[K:, :K]
//   V_{k+1} = [V* Q2] V_M[:, :K] = V* Z1 + W2 Z2,  Z2 = R2^{-1} V_M[K:, :K]
// Q1 and Q2 are never formed.
#include "launch.hpp"

namespace rpca {
namespace {

constexpr double JACOBI_EPS = 1e-15;
constexpr int JACOBI_MAX_SWEEPS = 40;
constexpr double CHOL_DEAD_REL = 1e-26;

// ---- helpers -----------------------------------------------------------------

template <int K>
__device__ inline void load_small(const double* __restrict__ g, double* s) {
    for (int e = threadIdx.x; e < K * K; e += blockDim.x) s[e] = g[(e / K) * KMAX + (e % K)];
}
template <int K>
__device__ inline void store_small(const double* s, double* __restrict__ g) {
    for (int e = threadIdx.x; e < K * K; e += blockDim.x) g[(e / K) * KMAX + (e % K)] = s[e];
}

// y = x A for a row vector x (1 x K) and A (K x K, ld K, LDS)
template <int K>
__device__ inline void rowmul(const double (&x)[K], const double* A, double (&y)[K]) {
#pragma unroll
    for (int j = 0; j < K; ++j) {
        double acc = 0.0;
#pragma unroll
        for (int i = 0; i < K; ++i) acc = fma(x[i], A[i * K + j], acc);
        y[j] = acc;
    }
}
// y = x A^T
template <int K>
__device__ inline void rowmul_t(const double (&x)[K], const double* A, double (&y)[K]) {
#pragma unroll
    for (int j = 0; j < K; ++j) {
        double acc = 0.0;
#pragma unroll
        for (int i = 0; i < K; ++i) acc = fma(x[i], A[j * K + i], acc);
        y[j] = acc;
    }
}

// Workgroup sum over threads of a (x) b -> dst[t1 * K + t2] (global, K*K entries).
// sa, sb: LDS scratch of PANEL_THREADS*K doubles each.
template <int K>
__device__ void block_outer_sum(const double (&a)[K], const double (&b)[K], double* sa, double* sb,
                                double* __restrict__ dst) {
#pragma unroll
    for (int t = 0; t < K; ++t) {
        sa[threadIdx.x * K + t] = a[t];
        sb[threadIdx.x * K + t] = b[t];
    }
    __syncthreads();
    for (int e = threadIdx.x; e < K * K; e += blockDim.x) {
        const int t1 = e / K, t2 = e % K;
        double acc = 0.0;
#pragma unroll 8
        for (int r = 0; r < PANEL_THREADS; ++r) acc = fma(sa[r * K + t1], sb[r * K + t2], acc);
        dst[e] = acc;
    }
    __syncthreads();
}

// Fixed-order sum of partial blocks [first, first+count) of gpart into s (LDS,
// K*K). Thread (e, g) sums the blocks b = g, g + G, ... of entry e with
// several loads in flight; the G group sums are then added in group order.
template <int K>
__device__ void sum_partials(const double* gpart, int first, int count, double* s) {
    constexpr int E = K * K;
    constexpr int G = PANEL_THREADS / E > 0 ? PANEL_THREADS / E : 1;
    __shared__ double tmp[G * E > PANEL_THREADS ? G * E : PANEL_THREADS];
    const int e = threadIdx.x % E, g = threadIdx.x / E;
    if (g < G) {
        double acc[4] = {0.0, 0.0, 0.0, 0.0};
        int b = g;
        for (; b + 3 * G < count; b += 4 * G) {
#pragma unroll
            for (int u = 0; u < 4; ++u) acc[u] += gpart[(size_t)(first + b + u * G) * KMAX * KMAX + e];
        }
        for (int u = 0; b < count; b += G, ++u) acc[u & 3] += gpart[(size_t)(first + b) * KMAX * KMAX + e];
        tmp[g * E + e] = (acc[0] + acc[1]) + (acc[2] + acc[3]);
    }
    __syncthreads();
    if (threadIdx.x < E) {
        double t = 0.0;
        for (int q = 0; q < G; ++q) t += tmp[q * E + threadIdx.x];
        s[threadIdx.x] = t;
    }
    __syncthreads();
}

// G = R^T R with R upper triangular (LDS, ld K), and Rinv = R^{-1}. A pivot
// that vanishes (d <= CHOL_DEAD_REL * G_jj or G_jj ~ 0) marks a numerically
// dependent column: its row of R and column of Rinv are set to zero.
template <int K>
__device__ void block_chol_inv(const double* G, double* R, double* Rinv) {
    for (int e = threadIdx.x; e < K * K; e += blockDim.x) { R[e] = 0.0; Rinv[e] = 0.0; }
    __syncthreads();
    for (int j = 0; j < K; ++j) {
        if (threadIdx.x == 0) {
            const double g = G[j * K + j];
            double d = g;
            for (int k = 0; k < j; ++k) d -= R[k * K + j] * R[k * K + j];
            const bool alive = g > 1e-300 && d > CHOL_DEAD_REL * g;
            R[j * K + j] = alive ? sqrt(d) : 0.0;
        }
        __syncthreads();
        const int c = threadIdx.x;
        if (c > j && c < K) {
            const double rjj = R[j * K + j];
            double v = 0.0;
            if (rjj != 0.0) {
                v = G[j * K + c];
                for (int k = 0; k < j; ++k) v -= R[k * K + j] * R[k * K + c];
                v /= rjj;
            }
            R[j * K + c] = v;
        }
        __syncthreads();
    }
    if (threadIdx.x < K) {
        const int c = threadIdx.x;
        double x[K];
        for (int i = K - 1; i >= 0; --i) {
            const double rii = R[i * K + i];
            double v = 0.0;
            if (rii != 0.0) {
                v = (i == c) ? 1.0 : 0.0;
                for (int k = i + 1; k < K; ++k) v -= R[i * K + k] * x[k];
                v /= rii;
            }
            x[i] = v;
        }
        for (int i = 0; i < K; ++i) Rinv[i * K + c] = x[i];
    }
    __syncthreads();
}

template <int CTRL> __device__ inline double dpp64(double x) {
    const int64_t u = __double_as_longlong(x);
    const int lo = __builtin_amdgcn_update_dpp(0, (int)(uint32_t)u, CTRL, 0xf, 0xf, true);
    const int hi = __builtin_amdgcn_update_dpp(0, (int)(uint32_t)(u >> 32), CTRL, 0xf, 0xf, true);
    return __longlong_as_double((int64_t)(((uint64_t)(uint32_t)hi << 32) | (uint32_t)lo));
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
// inner products. Sweeps stop when no pair needed a rotation
// (|a_p . a_q| <= JACOBI_EPS ||a_p|| ||a_q||). On return sig[] is descending
// and Uo/Vo hold left/right singular vectors as columns (column-major).
// Must be called by all 64 lanes of one wave; returns the sweep count.
template <int N>
__device__ int wave_jacobi_svd(double* A, double* V, double* sig, double* Uo, double* Vo) {
    static_assert(N % 2 == 0 && N <= 2 * KMAX, "even N up to 2*KMAX");
    constexpr int NP = N / 2;
    constexpr int LP0 = pow2_floor(WAVE / NP);
    constexpr int LP = LP0 > 16 ? 16 : LP0;
    constexpr int E = (N + LP - 1) / LP;
    const int lane = threadIdx.x & (WAVE - 1);
    for (int e = lane; e < N * N; e += WAVE) V[e] = ((e / N) == (e % N)) ? 1.0 : 0.0;
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
    const int q = lane / LP, g = lane % LP;
    int sweep = 0;
    for (; sweep < JACOBI_MAX_SWEEPS; ++sweep) {
        bool rotated = false;
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
                if (fabs(ga) > JACOBI_EPS * sqrt(al * be)) {
                    const double zt = (be - al) / (2.0 * ga);
                    const double t = fabs(zt) > 1e100 ? 0.5 / zt
                                                      : copysign(1.0, zt) / (fabs(zt) + sqrt(1.0 + zt * zt));
                    const double c = 1.0 / sqrt(1.0 + t * t);
                    const double s = c * t;
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
            __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
            __builtin_amdgcn_wave_barrier();
        }
        if (!__any(rotated)) break;
    }
    // column norms, ranks (descending, ties by index), normalised outputs
    if (lane < N) {
        const int j = lane;
        double acc = 0.0;
        for (int e = 0; e < N; ++e) acc = fma(A[j * N + e], A[j * N + e], acc);
        sig[j] = sqrt(acc);
    }
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
    double sj = 0.0;
    int rank = 0;
    if (lane < N) {
        sj = sig[lane];
        for (int i = 0; i < N; ++i) {
            const double si = sig[i];
            rank += (si > sj) || (si == sj && i < lane);
        }
    }
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
    if (lane < N) {
        sig[rank] = sj;
        const double inv = sj > 0.0 ? 1.0 / sj : 0.0;
        for (int e = 0; e < N; ++e) {
            Uo[rank * N + e] = A[lane * N + e] * inv;
            Vo[rank * N + e] = V[lane * N + e];
        }
    }
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
    return sweep + 1;
}

template <typename T> __device__ inline T* tptr(void* p) { return static_cast<T*>(p); }
template <typename T> __device__ inline const T* tptr(const void* p) { return static_cast<const T*>(p); }

__device__ inline void publish_status(const PanelArgs& a, const Ctrl* c) {
    if (a.host_status) {
        HostStatus st;
        st.seq = c->seq;
        st.done = c->done;
        st.stage = c->stage;
        st.k = c->k;
        st.err = c->err;
        st.zeta = c->zeta;
        *a.host_status = st;
        __threadfence_system();
    }
}

// ---- kernel 1: gather partial products, U_f^T Y1, residual, stopping rule ----

template <typename T, int K>
__global__ __launch_bounds__(PANEL_THREADS) void k_gather(PanelArgs a) {
    using Acc = typename AccOf<T>::type;
    constexpr int RPB = PANEL_THREADS / GATHER_SPLIT;   // rows per workgroup
    Ctrl* ctrl = a.ctrl;
    if (!body_runs(ctrl, a.body)) return;
    __shared__ double sa[PANEL_THREADS * K], sb[PANEL_THREADS * K];
    __shared__ double part[PANEL_THREADS * K];
    __shared__ int flag;
    const int gU = (a.m + RPB - 1) / RPB;
    const bool uside = (int)blockIdx.x < gU;
    const int lr = threadIdx.x % RPB, chunk = threadIdx.x / RPB;
    const int row = (uside ? blockIdx.x : blockIdx.x - gU) * RPB + lr;
    const int nrows = uside ? a.m : a.n;
    const int ntiles = uside ? a.n_ct : a.n_rt;
    const Acc* P = tptr<Acc>(uside ? a.P1 : a.P2);
    // this thread sums tiles c = chunk, chunk + SPLIT, ... of its row
    double y[K];
#pragma unroll
    for (int t = 0; t < K; ++t) y[t] = 0.0;
    if (row < nrows) {
        int c = chunk;
        for (; c + 3 * GATHER_SPLIT < ntiles; c += 4 * GATHER_SPLIT) {
            Acc v[4][K];
#pragma unroll
            for (int u = 0; u < 4; ++u)
#pragma unroll
                for (int t = 0; t < K; ++t) v[u][t] = P[((size_t)(c + u * GATHER_SPLIT) * nrows + row) * K + t];
#pragma unroll
            for (int u = 0; u < 4; ++u)
#pragma unroll
                for (int t = 0; t < K; ++t) y[t] += static_cast<double>(v[u][t]);
        }
        for (; c < ntiles; c += GATHER_SPLIT)
#pragma unroll
            for (int t = 0; t < K; ++t) y[t] += static_cast<double>(P[((size_t)c * nrows + row) * K + t]);
    }
#pragma unroll
    for (int t = 0; t < K; ++t) part[threadIdx.x * K + t] = y[t];
    __syncthreads();
    // chunk 0 adds the chunk sums in chunk order
    double uf[K];
#pragma unroll
    for (int t = 0; t < K; ++t) { uf[t] = 0.0; y[t] = 0.0; }
    if (chunk == 0 && row < nrows) {
        for (int q = 0; q < GATHER_SPLIT; ++q)
#pragma unroll
            for (int t = 0; t < K; ++t) y[t] += part[(q * RPB + lr) * K + t];
        double* Y = uside ? a.Y1 : a.Y2;
#pragma unroll
        for (int t = 0; t < K; ++t) Y[(size_t)row * K + t] = y[t];
        if (uside) {
            const T* Uf = tptr<T>(a.Uf);
#pragma unroll
            for (int t = 0; t < K; ++t) uf[t] = static_cast<double>(Uf[(size_t)row * K + t]);
        }
    }
    if (uside) block_outer_sum<K>(uf, y, sa, sb, a.gpart + (size_t)blockIdx.x * KMAX * KMAX);
    if (!last_block_arrives(&ctrl->cnt[CNT_GATHER], &flag)) return;

    // ---- last workgroup ----
    __shared__ double craw[K * K], ru[K * K], rv[K * K], tmp[K * K], red[4];
    sum_partials<K>(a.gpart, 0, gU, craw);
    load_small<K>(a.small->RUinv, ru);
    load_small<K>(a.small->RVinv, rv);
    __syncthreads();
    // C* = R_U^{-T} Craw R_V^{-1}
    for (int e = threadIdx.x; e < K * K; e += blockDim.x) {
        const int i = e / K, j = e % K;
        double acc = 0.0;
        for (int l = 0; l < K; ++l) acc = fma(craw[i * K + l], rv[l * K + j], acc);
        tmp[e] = acc;
    }
    __syncthreads();
    for (int e = threadIdx.x; e < K * K; e += blockDim.x) {
        const int i = e / K, j = e % K;
        double acc = 0.0;
        for (int l = 0; l < K; ++l) acc = fma(ru[l * K + i], tmp[l * K + j], acc);
        a.small->Cstar[i * KMAX + j] = acc;
    }
    double rs = 0.0;
    for (int b = threadIdx.x; b < a.n_tiles; b += blockDim.x) rs += __builtin_nontemporal_load(&a.resid[b]);
    rs = block_sum_256(rs, red);
    if (threadIdx.x == 0) {
        ctrl->resid2 = rs;
        if (ctrl->stage == STAGE_SIGMA_D) ctrl->normD2 = rs;   // zeta = +inf: the residual is ||D||_F^2
        if (ctrl->stage == STAGE_MAIN) {
            const double err = sqrt(rs / ctrl->normD2);
            ctrl->err = err;
            const int k = ctrl->k;
            if (a.err_hist && k < a.hist_cap) { a.err_hist[k] = err; a.zeta_hist[k] = ctrl->zeta; }
            if (ctrl->want_stop && (err < ctrl->tol || k >= ctrl->max_iter)) {
                ctrl->done = 1;
                ctrl->stopped_by_tol = err < ctrl->tol;
            }
        } else {
            ctrl->passes += 1;
            ctrl->total_passes += 1;
        }
        ctrl->active = ctrl->done ? 0 : 1;
        ctrl->seq += 1;
        ctrl->cnt[CNT_GATHER] = 0;
        publish_status(a, ctrl);
    }
}

// ---- kernel 2: complements W1, W2, their Grams, 2K x 2K SVD, threshold ------

template <typename T, int K>
__global__ __launch_bounds__(PANEL_THREADS) void k_complement(PanelArgs a) {
    constexpr int N = 2 * K;
    Ctrl* ctrl = a.ctrl;
    if (!ctrl->active) return;
    __shared__ double sa[PANEL_THREADS * K], sb[PANEL_THREADS * K];
    __shared__ double ru[K * K], rv[K * K], cs[K * K];
    __shared__ int flag;
    load_small<K>(a.small->RUinv, ru);
    load_small<K>(a.small->RVinv, rv);
    load_small<K>(a.small->Cstar, cs);
    __syncthreads();
    const bool uside = (int)blockIdx.x < a.gU;
    const int row = (uside ? blockIdx.x : blockIdx.x - a.gU) * PANEL_THREADS + threadIdx.x;
    double w[K];
#pragma unroll
    for (int t = 0; t < K; ++t) w[t] = 0.0;
    if (uside && row < a.m) {
        double uf[K], y[K], us[K], ys[K], uc[K];
        const T* Uf = tptr<T>(a.Uf);
#pragma unroll
        for (int t = 0; t < K; ++t) { uf[t] = static_cast<double>(Uf[(size_t)row * K + t]); y[t] = a.Y1[(size_t)row * K + t]; }
        rowmul<K>(uf, ru, us);     // U*_i
        rowmul<K>(y, rv, ys);      // (Z V*)_i
        rowmul<K>(us, cs, uc);     // U*_i C*
#pragma unroll
        for (int t = 0; t < K; ++t) { w[t] = ys[t] - uc[t]; a.W1[(size_t)row * K + t] = w[t]; }
    } else if (!uside && row < a.n) {
        double vf[K], y[K], vs[K], ys[K], vc[K];
        const T* Vf = tptr<T>(a.Vf);
#pragma unroll
        for (int t = 0; t < K; ++t) { vf[t] = static_cast<double>(Vf[(size_t)row * K + t]); y[t] = a.Y2[(size_t)row * K + t]; }
        rowmul<K>(vf, rv, vs);     // V*_j
        rowmul<K>(y, ru, ys);      // (Z^T U*)_j
        rowmul_t<K>(vs, cs, vc);   // V*_j C*^T
#pragma unroll
        for (int t = 0; t < K; ++t) { w[t] = ys[t] - vc[t]; a.W2[(size_t)row * K + t] = w[t]; }
    }
    block_outer_sum<K>(w, w, sa, sb, a.gpart + (size_t)blockIdx.x * KMAX * KMAX);
    if (!last_block_arrives(&ctrl->cnt[CNT_COMPLEMENT], &flag)) return;

    // ---- last workgroup: R1, R2, M, SVD(M), new coefficients, zeta ----
    __shared__ double g1[K * K], g2[K * K], r1[K * K], r1i[K * K], r2[K * K], r2i[K * K];
    __shared__ double Ma[N * N], Mv[N * N], Um[N * N], Vm[N * N], sg[N];
    __shared__ int sweeps;
    sum_partials<K>(a.gpart, 0, a.gU, g1);
    sum_partials<K>(a.gpart, a.gU, a.gV, g2);
    block_chol_inv<K>(g1, r1, r1i);
    block_chol_inv<K>(g2, r2, r2i);
    for (int e = threadIdx.x; e < N * N; e += blockDim.x) {
        const int col = e / N, rw = e % N;
        double v = 0.0;
        if (rw < K && col < K) v = cs[rw * K + col];
        else if (rw < K) v = r2[(col - K) * K + rw];          // R2^T
        else if (col < K) v = r1[(rw - K) * K + col];         // R1
        Ma[e] = v;
    }
    __syncthreads();
    if (threadIdx.x < WAVE) {
        const int sw = wave_jacobi_svd<N>(Ma, Mv, sg, Um, Vm);
        if (threadIdx.x == 0) sweeps = sw;
    }
    __syncthreads();
    Small* sm = a.small;
    for (int e = threadIdx.x; e < K * K; e += blockDim.x) {
        const int i = e / K, j = e % K;   // coefficient row i, singular triplet j
        double x2 = 0.0, z2 = 0.0;
        for (int l = 0; l < K; ++l) {
            x2 = fma(r1i[i * K + l], Um[j * N + K + l], x2);
            z2 = fma(r2i[i * K + l], Vm[j * N + K + l], z2);
        }
        sm->X1[i * KMAX + j] = Um[j * N + i];
        sm->X2[i * KMAX + j] = x2;
        sm->Z1[i * KMAX + j] = Vm[j * N + i];
        sm->Z2[i * KMAX + j] = z2;
    }
    if (threadIdx.x < N) sm->sigma_M[threadIdx.x] = sg[threadIdx.x];
    if (threadIdx.x < K) sm->sigma_new[threadIdx.x] = sg[threadIdx.x];
    if (threadIdx.x == 0) {
        const int r = ctrl->r;
        if (ctrl->stage == STAGE_MAIN) {
            // zeta_{k+1} = beta (sigma_{r+1} + gamma^{k+1} sigma_1)  (Algorithm 1)
            const int k = ctrl->k;
            const double s1 = sg[0], sr1 = sg[r];
            ctrl->sig1_pt = s1;
            ctrl->sigr1_pt = sr1;
            ctrl->zeta = ctrl->beta * (sr1 + pow(ctrl->gamma, (double)(k + 1)) * s1);
            ctrl->k = k + 1;
        } else {
            double acc = 0.0;
            for (int t = 0; t < r; ++t) acc += g1[t * K + t] + g2[t * K + t];
            const double res = sg[0] > 0.0 ? sqrt(acc) / sg[0] : 0.0;
            const double tolr = ctrl->stage == STAGE_SIGMA_D ? ctrl->tol_res_a : ctrl->tol_res_b;
            const bool conv = res <= tolr || (ctrl->passes >= 3 && res > 0.5 * ctrl->res_prev) ||
                              ctrl->passes >= ctrl->init_max_passes;
            ctrl->res_prev = res;
            if (conv && ctrl->stage == STAGE_SIGMA_D) {
                ctrl->sigma1_D = sg[0];
                ctrl->zeta = ctrl->beta_init * sg[0];     // zeta_{-1} = beta_init sigma_1(D)
                ctrl->stage = STAGE_INIT_Z;
                ctrl->passes = 0;
                ctrl->res_prev = 1e300;
            } else if (conv) {
                ctrl->zeta = ctrl->beta * sg[0];          // zeta_0 = beta sigma_1(D - S_{-1})
                ctrl->stage = STAGE_INIT_DONE;
            }
        }
        ctrl->jacobi_sweeps = sweeps;
        ctrl->cnt[CNT_COMPLEMENT] = 0;
        publish_status(a, ctrl);
    }
}

// ---- kernel 3: new factors (or entry from a given state), Trim, Gram(A) ------

template <typename T, int K>
__global__ __launch_bounds__(PANEL_THREADS) void k_update(PanelArgs a) {
    Ctrl* ctrl = a.ctrl;
    const bool from_m = a.mode == UPDATE_FROM_M;
    if (from_m && !ctrl->active) return;
    __shared__ double sa[PANEL_THREADS * K], sb[PANEL_THREADS * K];
    __shared__ double ru[K * K], rv[K * K], x1[K * K], x2[K * K], sig[K];
    __shared__ int flag;
    // Entering the loop (from a given state or from the initialisation) and
    // updates inside the loop produce an iterate L_k: rebuild factors + Trim.
    // Updates inside the initial subspace iteration only refresh the block.
    const bool main_stage = !from_m || ctrl->stage == STAGE_MAIN;
    if (from_m) {
        load_small<K>(a.small->RUinv, ru);
        load_small<K>(a.small->RVinv, rv);
    }
    const bool uside = (int)blockIdx.x < a.gU;
    if (from_m) load_small<K>(uside ? a.small->X1 : a.small->Z1, x1);
    if (from_m) load_small<K>(uside ? a.small->X2 : a.small->Z2, x2);
    if (threadIdx.x < K) sig[threadIdx.x] = from_m ? a.small->sigma_new[threadIdx.x] : (a.src_sigma ? a.src_sigma[threadIdx.x] : 1.0);
    __syncthreads();
    const int row = (uside ? blockIdx.x : blockIdx.x - a.gU) * PANEL_THREADS + threadIdx.x;
    const int nrows = uside ? a.m : a.n;
    double av[K];
#pragma unroll
    for (int t = 0; t < K; ++t) av[t] = 0.0;
    if (row < nrows) {
        double un[K];
        if (from_m) {
            const T* F = tptr<T>(uside ? a.Uf : a.Vf);
            const double* Wp = uside ? a.W1 : a.W2;
            double f[K], fs[K], w[K], p1[K], p2[K];
#pragma unroll
            for (int t = 0; t < K; ++t) { f[t] = static_cast<double>(F[(size_t)row * K + t]); w[t] = Wp[(size_t)row * K + t]; }
            rowmul<K>(f, uside ? ru : rv, fs);   // U*_i (or V*_j)
            rowmul<K>(fs, x1, p1);
            rowmul<K>(w, x2, p2);
#pragma unroll
            for (int t = 0; t < K; ++t) un[t] = p1[t] + p2[t];
        } else {
            const double* src = uside ? a.srcU : a.srcV;
#pragma unroll
            for (int t = 0; t < K; ++t) un[t] = src[(size_t)row * a.ld_src + t];
        }
        double* dst = uside ? a.Unew : a.Vnew;
        if (dst) {
#pragma unroll
            for (int t = 0; t < K; ++t) dst[(size_t)row * K + t] = un[t];
        }
        if (main_stage) {
            // rebuild factors of L: AL = U diag(sigma), BL = V
            T* LF = tptr<T>(uside ? a.AL : a.BL);
#pragma unroll
            for (int t = 0; t < K; ++t) LF[(size_t)row * K + t] = static_cast<T>(uside ? un[t] * sig[t] : un[t]);
        }
        // Algorithm 2: scale the row by min{1, c / ||row||}; c = sqrt(mu r / m) for U, sqrt(mu r / n) for V.
        double wgt = 1.0;
        if (main_stage && ctrl->trim) {
            double nr = 0.0;
#pragma unroll
            for (int t = 0; t < K; ++t) nr = fma(un[t], un[t], nr);
            nr = sqrt(nr);
            const double c = sqrt(ctrl->mu * (double)K / (double)(uside ? a.m : a.n));
            if (nr > c) wgt = c / nr;
        }
        double* Ap = uside ? a.Ap : a.Bp;
#pragma unroll
        for (int t = 0; t < K; ++t) { av[t] = wgt * un[t]; Ap[(size_t)row * K + t] = av[t]; }
    }
    block_outer_sum<K>(av, av, sa, sb, a.gpart + (size_t)blockIdx.x * KMAX * KMAX);
    if (!last_block_arrives(&ctrl->cnt[CNT_UPDATE], &flag)) return;

    __shared__ double g[K * K], rr[K * K], ri[K * K];
    sum_partials<K>(a.gpart, 0, a.gU, g);
    block_chol_inv<K>(g, rr, ri);
    store_small<K>(ri, a.small->RAinv);
    __syncthreads();
    sum_partials<K>(a.gpart, a.gU, a.gV, g);
    block_chol_inv<K>(g, rr, ri);
    store_small<K>(ri, a.small->RBinv);
    if (a.sigma_dst && threadIdx.x < K) a.sigma_dst[threadIdx.x] = sig[threadIdx.x];
    if (threadIdx.x == 0) {
        if (!from_m && ctrl->stage == STAGE_INIT_DONE) ctrl->stage = STAGE_MAIN;
        ctrl->cnt[CNT_UPDATE] = 0;
    }
}

// ---- kernel 4: orthonormal bases U~ = A R_A^{-1}, their dtype copies, Grams --

template <typename T, int K>
__global__ __launch_bounds__(PANEL_THREADS) void k_basis(PanelArgs a) {
    Ctrl* ctrl = a.ctrl;
    if (a.gated && !ctrl->active) return;
    __shared__ double sa[PANEL_THREADS * K], sb[PANEL_THREADS * K];
    __shared__ double ri[K * K];
    __shared__ int flag;
    const bool uside = (int)blockIdx.x < a.gU;
    load_small<K>(uside ? a.small->RAinv : a.small->RBinv, ri);
    __syncthreads();
    const int row = (uside ? blockIdx.x : blockIdx.x - a.gU) * PANEL_THREADS + threadIdx.x;
    const int nrows = uside ? a.m : a.n;
    double fv[K];
#pragma unroll
    for (int t = 0; t < K; ++t) fv[t] = 0.0;
    if (row < nrows) {
        const double* Ap = uside ? a.Ap : a.Bp;
        double av[K], q[K];
#pragma unroll
        for (int t = 0; t < K; ++t) av[t] = Ap[(size_t)row * K + t];
        rowmul<K>(av, ri, q);
        T* F = tptr<T>(uside ? a.Uf : a.Vf);
        double* out = uside ? a.outU : a.outV;
#pragma unroll
        for (int t = 0; t < K; ++t) {
            const T qt = static_cast<T>(q[t]);
            F[(size_t)row * K + t] = qt;
            fv[t] = static_cast<double>(qt);
            if (out) out[(size_t)row * K + t] = q[t];
        }
    }
    block_outer_sum<K>(fv, fv, sa, sb, a.gpart + (size_t)blockIdx.x * KMAX * KMAX);
    if (!last_block_arrives(&ctrl->cnt[CNT_BASIS], &flag)) return;

    __shared__ double g[K * K], rr[K * K], rinv[K * K];
    sum_partials<K>(a.gpart, 0, a.gU, g);
    block_chol_inv<K>(g, rr, rinv);
    store_small<K>(rinv, a.small->RUinv);
    __syncthreads();
    sum_partials<K>(a.gpart, a.gU, a.gV, g);
    block_chol_inv<K>(g, rr, rinv);
    store_small<K>(rinv, a.small->RVinv);
    if (threadIdx.x == 0) ctrl->cnt[CNT_BASIS] = 0;
}

// ---- start block of the initial subspace iteration ---------------------------

__device__ inline double hash_uniform(uint64_t seed, uint64_t idx) {
    // splitmix64 of (seed, idx) -> uniform in [-1, 1)
    uint64_t z = seed + 0x9E3779B97F4A7C15ull * (idx + 1);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    z = z ^ (z >> 31);
    return (double)(z >> 11) * (2.0 / 9007199254740992.0) - 1.0;
}

template <int K>
__global__ __launch_bounds__(PANEL_THREADS) void k_start(PanelArgs a) {
    Ctrl* ctrl = a.ctrl;
    __shared__ double sa[PANEL_THREADS * K], sb[PANEL_THREADS * K];
    __shared__ int flag;
    const bool uside = (int)blockIdx.x < a.gU;
    const int row = (uside ? blockIdx.x : blockIdx.x - a.gU) * PANEL_THREADS + threadIdx.x;
    const int nrows = uside ? a.m : a.n;
    double av[K];
#pragma unroll
    for (int t = 0; t < K; ++t) av[t] = 0.0;
    if (row < nrows) {
        double* Ap = uside ? a.Ap : a.Bp;
        const uint64_t base = (uside ? 0ull : (uint64_t)a.m * K) + (uint64_t)row * K;
#pragma unroll
        for (int t = 0; t < K; ++t) { av[t] = hash_uniform(a.seed, base + t); Ap[(size_t)row * K + t] = av[t]; }
    }
    block_outer_sum<K>(av, av, sa, sb, a.gpart + (size_t)blockIdx.x * KMAX * KMAX);
    if (!last_block_arrives(&ctrl->cnt[CNT_START], &flag)) return;
    __shared__ double g[K * K], rr[K * K], ri[K * K];
    sum_partials<K>(a.gpart, 0, a.gU, g);
    block_chol_inv<K>(g, rr, ri);
    store_small<K>(ri, a.small->RAinv);
    __syncthreads();
    sum_partials<K>(a.gpart, a.gU, a.gV, g);
    block_chol_inv<K>(g, rr, ri);
    store_small<K>(ri, a.small->RBinv);
    if (threadIdx.x == 0) ctrl->cnt[CNT_START] = 0;
}

__global__ void k_setup(Ctrl* ctrl, Ctrl init) { if (threadIdx.x == 0 && blockIdx.x == 0) *ctrl = init; }

template <typename T>
__global__ void k_convert(const double* __restrict__ src, T* __restrict__ dst, int64_t count,
                          const double* __restrict__ scale, int K) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < count) dst[i] = static_cast<T>(scale ? src[i] * scale[i % K] : src[i]);
}

#define RPCA_K_SWITCH(CALL)                                                                      \
    switch (K) {                                                                                 \
        case 1: CALL(1); break; case 2: CALL(2); break; case 3: CALL(3); break;                  \
        case 4: CALL(4); break; case 5: CALL(5); break; case 6: CALL(6); break;                  \
        case 7: CALL(7); break; case 8: CALL(8); break; case 9: CALL(9); break;                  \
        case 10: CALL(10); break; case 11: CALL(11); break; case 12: CALL(12); break;            \
        case 13: CALL(13); break; case 14: CALL(14); break; case 15: CALL(15); break;            \
        case 16: CALL(16); break;                                                                \
        default: return hipErrorInvalidValue;                                                    \
    }

}  // namespace

#define RPCA_LAUNCH_F(KK) hipLaunchKernelGGL((KFUN<float, KK>), grid, block, 0, s, a)
#define RPCA_LAUNCH_D(KK) hipLaunchKernelGGL((KFUN<double, KK>), grid, block, 0, s, a)

#define KFUN k_gather
hipError_t launch_gather(const PanelArgs& a, int K, int dtype, hipStream_t s) {
    constexpr int RPB = PANEL_THREADS / GATHER_SPLIT;
    const dim3 grid((unsigned)((a.m + RPB - 1) / RPB + (a.n + RPB - 1) / RPB)), block(PANEL_THREADS);
    if (dtype == 1) { RPCA_K_SWITCH(RPCA_LAUNCH_F) } else { RPCA_K_SWITCH(RPCA_LAUNCH_D) }
    return hipGetLastError();
}
#undef KFUN
#define KFUN k_complement
hipError_t launch_complement(const PanelArgs& a, int K, int dtype, hipStream_t s) {
    const dim3 grid((unsigned)(a.gU + a.gV)), block(PANEL_THREADS);
    if (dtype == 1) { RPCA_K_SWITCH(RPCA_LAUNCH_F) } else { RPCA_K_SWITCH(RPCA_LAUNCH_D) }
    return hipGetLastError();
}
#undef KFUN
#define KFUN k_update
hipError_t launch_update(const PanelArgs& a, int K, int dtype, hipStream_t s) {
    const dim3 grid((unsigned)(a.gU + a.gV)), block(PANEL_THREADS);
    if (dtype == 1) { RPCA_K_SWITCH(RPCA_LAUNCH_F) } else { RPCA_K_SWITCH(RPCA_LAUNCH_D) }
    return hipGetLastError();
}
#undef KFUN
#define KFUN k_basis
hipError_t launch_basis(const PanelArgs& a, int K, int dtype, hipStream_t s) {
    const dim3 grid((unsigned)(a.gU + a.gV)), block(PANEL_THREADS);
    if (dtype == 1) { RPCA_K_SWITCH(RPCA_LAUNCH_F) } else { RPCA_K_SWITCH(RPCA_LAUNCH_D) }
    return hipGetLastError();
}
#undef KFUN

#define RPCA_LAUNCH_START(KK) hipLaunchKernelGGL((k_start<KK>), grid, block, 0, s, a)
hipError_t launch_start(const PanelArgs& a, int K, hipStream_t s) {
    const dim3 grid((unsigned)(a.gU + a.gV)), block(PANEL_THREADS);
    RPCA_K_SWITCH(RPCA_LAUNCH_START)
    return hipGetLastError();
}

hipError_t launch_setup(Ctrl* ctrl, const Ctrl& init, hipStream_t s) {
    hipLaunchKernelGGL(k_setup, dim3(1), dim3(64), 0, s, ctrl, init);
    return hipGetLastError();
}

hipError_t launch_convert(const double* src, void* dst, int64_t count, const double* scale, int K, int dtype,
                          hipStream_t s) {
    if (count <= 0) return hipSuccess;
    const dim3 grid((unsigned)((count + 255) / 256)), block(256);
    if (dtype == 1) hipLaunchKernelGGL(k_convert<float>, grid, block, 0, s, src, static_cast<float*>(dst), count, scale, K);
    else hipLaunchKernelGGL(k_convert<double>, grid, block, 0, s, src, static_cast<double*>(dst), count, scale, K);
    return hipGetLastError();
}

}  // namespace rpca
