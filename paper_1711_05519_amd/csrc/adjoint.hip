// Reverse mode of K unrolled relaxed iterations (training of a threshold
// schedule; not part of the paper).
//
// One relaxed body from L_k = U diag(sigma) V^T (Algorithm 1 with the hard
// threshold replaced by s(x) = x logistic((|x| - zeta) / tau)):
//   Trim (Algorithm 2): A = diag(w_U) U, B = diag(w_V) V; U~ = A R_A^{-1},
//   V~ = B R_B^{-1} (Cholesky QR);  X = D - L_k,  Z = D - s(X);
//   Y1 = Z V~, Y2 = Z^T U~, C = U~^T Y1, W1 = Y1 - U~ C = Q1 R1, W2 = Y2 - V~ V~^T Y2 = Q2 R2;
//   M = [[C, R2^T], [R1, 0]] = U_M S V_M^T;  L_{k+1} = H_r(P_T(Z)) = B_U H_r(M) B_V^T,
//   B_U = [U~ Q1], B_V = [V~ Q2]   (Section 2.1).
// The loss is sum_k w_k ||L_k - P Q^T||_F^2 / ||P Q^T||_F^2 over the iterates.
//
// Between bodies the gradient is taken with respect to L_k (the next body
// depends on the factors only through L_k and its spans), and it is never
// formed: it is Lbar_k = Zbar_k o s'(X_k) + F1 V^T + U F2^T (o the entrywise
// product), with the tangent-space matrix Zbar_k = U~ X_^T + Y_ V~^T. Body k's
// reverse step needs only Gamma_V = Lbar_{k+1} B_V and Gamma_U = Lbar_{k+1}^T B_U
// (thin), which the previous reverse step forms while it streams over D. Per
// body, with Mhat = B_U^T Gamma_V:
//   H_r:  Ybar = B_U Kc B_V^T + Gt_V Pi_V B_V^T + B_U Pi_U Gt_U^T,
//         Kc = U_M Phi(U_M^T Mhat V_M) V_M^T (Phi: the first-order coefficients
//         of the top-r singular triplets, a symmetric map), Pi_U = U_M,r U_M,r^T,
//         Pi_V = V_M,r V_M,r^T, Gt_V = Gamma_V - B_U Mhat, Gt_U = Gamma_U - B_V Mhat^T;
//   P_T:  Zbar = P_T(Ybar) = U~ X_^T + Y_ V~^T, and for the projectors
//         G_U = (Pbar_U + Pbar_U^T) U~ = (B_U Kc[:, r:] + Gt_V Pi_V[:, r:]) R2 + Z N_V,
//         G_V = (B_V Kc[r:, :]^T + Gt_U Pi_U[:, r:]) R1 + Z^T N_U,
//         N_V = (I - P_V) Ybar^T U~, N_U = (I - P_U) Ybar V~ = Y_;
//   QR:   Abar = (I - P_U) G_U R_A^{-T};  Trim: Ubar_i = w_i Abar_i - [|U_i| > c] (c/|U_i|^3)(Abar_i . U_i) U_i;
//   s:    dloss/dzeta_k = sum Zbar o X g (1 - g) / tau;  dZ/dL = s'(X) = g + |X| g (1 - g) / tau;
//   to L_k: F1 = (I - U U^T) Ubar_trim Sigma^{-1}, F2 = (I - V V^T) Vbar_trim Sigma^{-1}.
// At the first body the gradients with respect to the free factors are
// returned: Ubar_0 = (Zbar o s') V Sigma + Ubar_trim, Vbar_0 likewise,
// sigmabar_t = U_t^T (Zbar o s') V_t.
//
// Kernels: a pass over D per body and direction (recompute of Y1, Y2; then
// Z N_V, Z^T N_U, the zeta derivative and the Hadamard products with the
// previous body's bases), thin Grams summed in a fixed order, thin row
// combinations out = [panels] S with S formed by single-wave FP64 tails, and
// the row-local Trim steps. Everything but D is FP64.

#include <string.h>

#include "../../include/rpca.h"
#include "launch.hpp"
#include "wave.hpp"

namespace rpca {
namespace {

constexpr int AJ_ROWS = 64;       // rows per workgroup of a Gram
constexpr int AJ_GW = 80;         // widest row of a Gram's two concatenated panels
constexpr int AJ_GE = 2048;       // entries of a Gram partial (and of a small-matrix slot)
constexpr int AJ_NPAN = 4;        // panels per side of a Gram or per combination

struct PanelRef {
    const double* p;
    int32_t ld, w;
};

struct GramJob {
    PanelRef L[AJ_NPAN], R[AJ_NPAN];
    int32_t nL, nR, wL, wR, rows;
    double* out;                  // wL x wR, row-major
};

struct GramArgs {
    GramJob job[2];
    int32_t nblk[2];
    double* gpart;
    uint32_t* cnt;
};

struct CombJob {
    PanelRef in[AJ_NPAN];
    int32_t nin, win, rows, q;
    const double* S;              // win x q, row-major
    double* out;
    int32_t ldo;
};

struct CombArgs {
    CombJob job[2];
    int32_t nblk[2];
};

__device__ inline double panel_get(const PanelRef* P, int np, int row, int c) {
    for (int q = 0; q < np; ++q) {
        if (c < P[q].w) return P[q].p[(size_t)row * P[q].ld + c];
        c -= P[q].w;
    }
    return 0.0;
}

// ---- thin Grams: out = [L panels]^T [R panels] over the rows, two jobs per launch
__global__ __launch_bounds__(256) void k_adj_gram(GramArgs g) {
    const int jb = (int)blockIdx.x < g.nblk[0] ? 0 : 1;
    const int b = jb ? (int)blockIdx.x - g.nblk[0] : (int)blockIdx.x;
    const GramJob& J = g.job[jb];
    __shared__ double rows[AJ_ROWS][AJ_GW + 1];
    const int W = J.wL + J.wR;
    const int r0 = b * AJ_ROWS;
    for (int e = threadIdx.x; e < AJ_ROWS * W; e += 256) {
        const int rr = e / W, c = e - rr * W, row = r0 + rr;
        double v = 0.0;
        if (row < J.rows) v = c < J.wL ? panel_get(J.L, J.nL, row, c) : panel_get(J.R, J.nR, row, c - J.wL);
        rows[rr][c] = v;
    }
    __syncthreads();
    double* gp = g.gpart + (size_t)blockIdx.x * AJ_GE;
    const int E = J.wL * J.wR;
    for (int e = threadIdx.x; e < E; e += 256) {
        const int i = e / J.wR, j = e - i * J.wR;
        double v = 0.0;
        for (int rr = 0; rr < AJ_ROWS; ++rr) v = fma(rows[rr][i], rows[rr][J.wL + j], v);
        gp[e] = v;
    }
    __shared__ int flag;
    if (!last_block_arrives(g.cnt, &flag)) return;
    for (int jj = 0; jj < 2; ++jj) {
        const GramJob& Q = g.job[jj];
        const int first = jj ? g.nblk[0] : 0, count = g.nblk[jj];
        const int EQ = Q.wL * Q.wR;
        for (int e = threadIdx.x; e < EQ; e += 256) {
            double v = 0.0;
            for (int bb = 0; bb < count; ++bb) v += g.gpart[(size_t)(first + bb) * AJ_GE + e];
            Q.out[e] = v;
        }
    }
    if (threadIdx.x == 0) *g.cnt = 0;
}

// ---- thin row combinations: out[i][c] = sum_t in(i, t) S[t][c], one thread per entry
__global__ __launch_bounds__(256) void k_adj_combine(CombArgs a) {
    const int jb = (int)blockIdx.x < a.nblk[0] ? 0 : 1;
    const int b = jb ? (int)blockIdx.x - a.nblk[0] : (int)blockIdx.x;
    const CombJob& J = a.job[jb];
    __shared__ double S[AJ_GE];
    for (int e = threadIdx.x; e < J.win * J.q; e += 256) S[e] = J.S[e];
    __syncthreads();
    const int64_t idx = (int64_t)b * 256 + threadIdx.x;
    if (idx >= (int64_t)J.rows * J.q) return;
    const int row = (int)(idx / J.q), c = (int)(idx - (int64_t)row * J.q);
    double v = 0.0;
    int off = 0;
    for (int q = 0; q < J.nin; ++q) {
        const double* src = J.in[q].p + (size_t)row * J.in[q].ld;
        for (int t = 0; t < J.in[q].w; ++t) v = fma(src[t], S[(off + t) * J.q + c], v);
        off += J.in[q].w;
    }
    J.out[(size_t)row * J.ldo + c] = v;
}

// ---- Trim, row by row (both sides in one launch) ----------------------------------
struct TrimArgs {
    const double* X[2];     // U (m x K), V (n x K)
    double* A[2];           // diag(w) X
    double* w[2];
    double* rho[2];
    const double* Abar[2];  // reverse: gradient of A
    double* Xbar[2];        // reverse: gradient of X
    double c[2];            // trim levels; <= 0 without trim
    int32_t rows[2], nblk0, K;
};

__global__ __launch_bounds__(256) void k_adj_trim(TrimArgs a, int reverse) {
    const int side = (int)blockIdx.x < a.nblk0 ? 0 : 1;
    const int row = (side ? (int)blockIdx.x - a.nblk0 : (int)blockIdx.x) * 256 + threadIdx.x;
    if (row >= a.rows[side]) return;
    const int K = a.K;
    const double* x = a.X[side] + (size_t)row * K;
    double rr = 0.0;
    for (int t = 0; t < K; ++t) rr = fma(x[t], x[t], rr);
    const double rho = sqrt(rr), c = a.c[side];
    const bool big = c > 0.0 && rho > c;
    const double w = big ? c / rho : 1.0;
    if (!reverse) {
        for (int t = 0; t < K; ++t) a.A[side][(size_t)row * K + t] = w * x[t];
        a.w[side][row] = w;
        a.rho[side][row] = rho;
        return;
    }
    const double* ab = a.Abar[side] + (size_t)row * K;
    double dot = 0.0;
    for (int t = 0; t < K; ++t) dot = fma(ab[t], x[t], dot);
    const double f = big ? c / (rho * rho * rho) * dot : 0.0;
    for (int t = 0; t < K; ++t) a.Xbar[side][(size_t)row * K + t] = fma(w, ab[t], -f * x[t]);
}

// ---- the pass over D ----------------------------------------------------------------
//
// Tile TM x 256, one thread per column. Per element: x = D - L_k, g, z = D - s(x),
// and (reverse) zd = x g (1 - g) / tau, s' = g + |x| g (1 - g) / tau,
// Zbar = Uz_i . Xz_j + Yz_i . Vz_j, h = Zbar s'. Row products
// [z ro0_j | h ro1_j] are summed over the tile's columns (wave shuffles, then
// the waves in order), column products [z co0_i | h co1_i] over its rows in
// registers. Per tile: sum (x - s)^2 and sum Zbar zd.
struct AdjStream {
    const void* D;
    int64_t ldd;
    int32_t m, n, TM, n_ct, n_rt, hw;
    const double* U;
    const double* sig;
    const double* V;
    double zeta, tau;
    PanelRef ro0, ro1, co0, co1;
    PanelRef Uz, Yz, Xz, Vz;
    double* Rp;       // [n_ct][m][WR]
    double* Cp;       // [n_rt][n][WC]
    double* scal;     // [tiles][2]
};

__device__ inline double logistic(double u) { return 0.5 * (1.0 + tanh(0.5 * u)); }

template <typename T, int K, bool BWD>
__global__ __launch_bounds__(RX_THREADS) void k_adj_stream(AdjStream a) {
    constexpr int W2 = BWD ? 2 * K : 0;
    constexpr int KZ = BWD ? K : 1;
    const int WR = K + (BWD ? a.hw : 0);
    const int lane = threadIdx.x & (WAVE - 1), wave = threadIdx.x / WAVE;
    const int ct = blockIdx.x % a.n_ct, rt = blockIdx.x / a.n_ct;
    const int j = ct * RX_THREADS + threadIdx.x;
    const bool valid = j < a.n;
    const int i_lo = rt * a.TM, i_hi = min(a.m, i_lo + a.TM);
    const T* __restrict__ D = static_cast<const T*>(a.D);
    const double zeta = a.zeta, tau = a.tau;
    double vb[K], ro[K + W2], acc[K + W2], xz[KZ], vz[KZ];
#pragma unroll
    for (int t = 0; t < K; ++t) {
        vb[t] = valid ? a.V[(size_t)j * K + t] : 0.0;
        ro[t] = valid ? a.ro0.p[(size_t)j * a.ro0.ld + t] : 0.0;
    }
#pragma unroll
    for (int t = 0; t < W2; ++t) ro[K + t] = (valid && t < a.hw) ? a.ro1.p[(size_t)j * a.ro1.ld + t] : 0.0;
#pragma unroll
    for (int t = 0; t < K + W2; ++t) acc[t] = 0.0;
    if constexpr (BWD) {
#pragma unroll
        for (int t = 0; t < K; ++t) {
            xz[t] = valid ? a.Xz.p[(size_t)j * a.Xz.ld + t] : 0.0;
            vz[t] = valid ? a.Vz.p[(size_t)j * a.Vz.ld + t] : 0.0;
        }
    }
    __shared__ double red[RX_THREADS / WAVE][3 * RX_KMAX];
    __shared__ double bred[RX_THREADS / WAVE];
    double res = 0.0, zsum = 0.0;
    for (int i = i_lo; i < i_hi; ++i) {
        double x = valid ? static_cast<double>(D[(size_t)i * a.ldd + j]) : 0.0;
        const double d = x;
#pragma unroll
        for (int t = 0; t < K; ++t) x = fma(-(a.U[(size_t)i * K + t] * a.sig[t]), vb[t], x);
        const double g = logistic((fabs(x) - zeta) / tau);
        const double s = x * g;
        const double z = valid ? d - s : 0.0;
        double h = 0.0;
        if (valid) res = fma(x - s, x - s, res);
        if constexpr (BWD) {
            double zb = 0.0;
#pragma unroll
            for (int t = 0; t < K; ++t) {
                zb = fma(a.Uz.p[(size_t)i * a.Uz.ld + t], xz[t], zb);
                zb = fma(a.Yz.p[(size_t)i * a.Yz.ld + t], vz[t], zb);
            }
            const double gg = g * (1.0 - g) / tau;
            if (valid) {
                zsum = fma(zb, x * gg, zsum);
                h = zb * fma(fabs(x), gg, g);
            }
        }
#pragma unroll
        for (int t = 0; t < K; ++t) acc[t] = fma(z, a.co0.p[(size_t)i * a.co0.ld + t], acc[t]);
        if constexpr (BWD) {
#pragma unroll
            for (int t = 0; t < W2; ++t)
                if (t < a.hw) acc[K + t] = fma(h, a.co1.p[(size_t)i * a.co1.ld + t], acc[K + t]);
        }
#pragma unroll
        for (int t = 0; t < K + W2; ++t) {
            if (t < WR) {
                double v = (t < K ? z : h) * ro[t];
                for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, WAVE);
                if (lane == 0) red[wave][t] = v;
            }
        }
        __syncthreads();
        if ((int)threadIdx.x < WR) {
            double v = 0.0;
            for (int w = 0; w < RX_THREADS / WAVE; ++w) v += red[w][threadIdx.x];
            a.Rp[((size_t)ct * a.m + i) * WR + threadIdx.x] = v;
        }
        __syncthreads();
    }
    if (valid) {
#pragma unroll
        for (int t = 0; t < K + W2; ++t)
            if (t < WR) a.Cp[((size_t)rt * a.n + j) * WR + t] = acc[t];
    }
    const double r1 = block_sum(res, bred);
    const double r2 = block_sum(zsum, bred);
    if (threadIdx.x == 0) {
        a.scal[2 * blockIdx.x] = r1;
        a.scal[2 * blockIdx.x + 1] = r2;
    }
}

// Sums of the pass's tile partials, in tile order: SR = sum_ct Rp (m x W),
// SC = sum_rt Cp (n x W); block 0 also sums the per-tile scalars.
struct SumArgs {
    const double* Rp;
    const double* Cp;
    const double* scal;
    double* SR;
    double* SC;
    double* scal_out;
    int32_t m, n, W, n_ct, n_rt;
};

__global__ __launch_bounds__(256) void k_adj_sum(SumArgs a) {
    const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
    const int64_t mW = (int64_t)a.m * a.W, nW = (int64_t)a.n * a.W;
    if (e < mW) {
        double v = 0.0;
        for (int c = 0; c < a.n_ct; ++c) v += a.Rp[(size_t)c * mW + e];
        a.SR[e] = v;
    } else if (e < mW + nW) {
        const int64_t f = e - mW;
        double v = 0.0;
        for (int r = 0; r < a.n_rt; ++r) v += a.Cp[(size_t)r * nW + f];
        a.SC[f] = v;
    }
    if (blockIdx.x == 0 && threadIdx.x < 2) {
        double v = 0.0;
        for (int b = 0; b < a.n_ct * a.n_rt; ++b) v += a.scal[2 * b + threadIdx.x];
        a.scal_out[threadIdx.x] = v;
    }
}

// ---- single-wave FP64 tails ---------------------------------------------------------
//
// Small matrices are row-major unless stated; the SVD of M keeps the
// column-major layout of the Jacobi routine (vector b in entries b N .. b N + N - 1).
struct TailArgs {
    const double* in[6];
    double* out[6];
    double c;       // loss coefficient 2 w / ||P Q^T||^2 (without the division)
    int32_t rt;     // rank of the target factors
    int32_t init;   // gamma tail: the first reverse step (no H, F panels)
};

template <int K>
__device__ void tail_chol(const TailArgs& a) {
    // in[0], in[1]: K x K Grams (U side, V side) -> out[0], out[1]: R^{-1};
    // out[2], out[3]: R (when given)
    __shared__ double G0[K * K], G1[K * K], R0[K * K], R1[K * K], I0[K * K], I1[K * K];
    const int lane = lane_id();
    for (int e = lane; e < K * K; e += WAVE) {
        G0[e] = a.in[0][e];
        G1[e] = a.in[1][e];
    }
    wave_sync();
    w_chol_inv2<K>(G0, R0, I0, G1, R1, I1);
    wave_sync();
    for (int e = lane; e < K * K; e += WAVE) {
        a.out[0][e] = I0[e];
        a.out[1][e] = I1[e];
        if (a.out[2]) a.out[2][e] = R0[e];
        if (a.out[3]) a.out[3][e] = R1[e];
    }
}

// in[0] = U~^T Y1, in[1] = V~^T Y2 (K x K) -> out[0] = [[I], [-C]], out[1] = [[I], [-C2]] (2K x K); out[2] = C
template <int K>
__device__ void tail_c(const TailArgs& a) {
    const int lane = lane_id();
    for (int e = lane; e < 2 * K * K; e += WAVE) {
        const int r = e / K, c = e % K;
        const double id = (r == c) ? 1.0 : 0.0;
        a.out[0][e] = r < K ? id : -a.in[0][(r - K) * K + c];
        a.out[1][e] = r < K ? id : -a.in[1][(r - K) * K + c];
    }
    for (int e = lane; e < K * K; e += WAVE) a.out[2][e] = a.in[0][e];
}

// in[0] = C, in[1] = R1, in[2] = R2 -> out[0] = U_M, out[1] = S, out[2] = V_M
// (column-major 2K x 2K)
template <int K>
__device__ void tail_m(const TailArgs& a) {
    constexpr int N = 2 * K;
    __shared__ double Mm[N * N], Vw[N * N], Uo[N * N], Vo[N * N], sg[N];
    const int lane = lane_id();
    // M = [[C, R2^T], [R1, 0]], column-major: element (row, col) at col * N + row
    for (int e = lane; e < N * N; e += WAVE) {
        const int col = e / N, row = e % N;
        double v = 0.0;
        if (row < K && col < K) v = a.in[0][row * K + col];
        else if (row < K) v = a.in[2][(col - K) * K + row];
        else if (col < K) v = a.in[1][(row - K) * K + col];
        Mm[e] = v;
    }
    wave_sync();
    wave_jacobi_svd<N, false>(Mm, Vw, sg, Uo, Vo);
    for (int e = lane; e < N * N; e += WAVE) {
        a.out[0][e] = Uo[e];
        a.out[2][e] = Vo[e];
    }
    if (lane < N) a.out[1][lane] = sg[lane];
}

// Reverse step of H_r. in[0] = Mhat = B_U^T Gamma_V (2K x 2K row-major),
// in[1] = U_M, in[2] = S, in[3] = V_M (column-major), in[4] = R1, in[5] = R2.
// out[0] = S_U (4K x 2K): [Y_ | GU0] = [B_U | Gamma_V] S_U;
// out[1] = S_V (4K x 3K): [X_ | N_V | GV0] = [B_V | Gamma_U] S_V.
template <int K>
__device__ void tail_b2(const TailArgs& a) {
    constexpr int N = 2 * K;
    __shared__ double Mh[N * N], Um[N * N], Vm[N * N], sg[N], E[N * N], F[N * N], T1[N * N], Kc[N * N];
    __shared__ double PU[N * N], PV[N * N], A1[N * N], A2[N * N], Tn[N * K];
    const int lane = lane_id();
    for (int e = lane; e < N * N; e += WAVE) {
        Mh[e] = a.in[0][e];
        Um[e] = a.in[1][e];
        Vm[e] = a.in[3][e];
    }
    if (lane < N) sg[lane] = a.in[2][lane];
    wave_sync();
    // singular vectors of negligible singular values are not defined by the
    // one-sided method: drop them (their part enters through the projector term)
    const double cut = 1e-12 * sg[0];
    for (int e = lane; e < N * N; e += WAVE)
        if (!(sg[e / N] > cut)) Um[e] = 0.0;
    wave_sync();
    // T1 = Mhat V_M (row-major), E = U_M^T T1
    for (int e = lane; e < N * N; e += WAVE) {
        const int r = e / N, b = e % N;
        double v = 0.0;
        for (int c = 0; c < N; ++c) v = fma(Mh[r * N + c], Vm[b * N + c], v);
        T1[e] = v;
    }
    wave_sync();
    for (int e = lane; e < N * N; e += WAVE) {
        const int i = e / N, j = e % N;
        double v = 0.0;
        for (int r = 0; r < N; ++r) v = fma(Um[i * N + r], T1[r * N + j], v);
        E[e] = v;
    }
    wave_sync();
    for (int e = lane; e < N * N; e += WAVE) {
        const int i = e / N, j = e % N;
        double f = 0.0;
        if (i < K && j < K) {
            f = E[e];
        } else if (i < K) {
            const double si = sg[i], sj = sg[j];
            f = (si * si * E[i * N + j] + si * sj * E[j * N + i]) / (si * si - sj * sj);
        } else if (j < K) {
            const double si = sg[j], sj = sg[i];
            f = (si * si * E[i * N + j] + si * sj * E[j * N + i]) / (si * si - sj * sj);
        }
        F[e] = f;
    }
    wave_sync();
    // Kc = U_M F V_M^T + (I - U_M U_M^T) Mhat V_M,K V_M,K^T (the dropped left vectors)
    for (int e = lane; e < N * K; e += WAVE) {
        const int r = e / K, t = e % K;   // Tn = (I - U U^T) Mhat V_K, N x K
        double v = T1[r * N + t];
        for (int b = 0; b < N; ++b) {
            double ub = 0.0;
            for (int c = 0; c < N; ++c) ub = fma(Um[b * N + c], T1[c * N + t], ub);
            v = fma(-Um[b * N + r], ub, v);
        }
        Tn[e] = v;
    }
    for (int e = lane; e < N * N; e += WAVE) {   // A1 = U_M F (row-major)
        const int r = e / N, j = e % N;
        double v = 0.0;
        for (int i = 0; i < N; ++i) v = fma(Um[i * N + r], F[i * N + j], v);
        A1[e] = v;
    }
    wave_sync();
    for (int e = lane; e < N * N; e += WAVE) {
        const int r = e / N, c = e % N;
        double v = 0.0;
        for (int j = 0; j < N; ++j) v = fma(A1[r * N + j], Vm[j * N + c], v);
        for (int t = 0; t < K; ++t) v = fma(Tn[r * K + t], Vm[t * N + c], v);
        Kc[e] = v;
        double pu = 0.0, pv = 0.0;
        for (int t = 0; t < K; ++t) {
            pu = fma(Um[t * N + r], Um[t * N + c], pu);
            pv = fma(Vm[t * N + r], Vm[t * N + c], pv);
        }
        PU[e] = pu;
        PV[e] = pv;
    }
    wave_sync();
    // A1 = Mhat Pi_V, A2 = Mhat^T Pi_U (row-major N x N)
    for (int e = lane; e < N * N; e += WAVE) {
        const int r = e / N, c = e % N;
        double v1 = 0.0, v2 = 0.0;
        for (int l = 0; l < N; ++l) {
            v1 = fma(Mh[r * N + l], PV[l * N + c], v1);
            v2 = fma(Mh[l * N + r], PU[l * N + c], v2);
        }
        A1[e] = v1;
        A2[e] = v2;
    }
    wave_sync();
    const double* R1 = a.in[4];
    const double* R2 = a.in[5];
    // S_U rows 0..N-1 (B_U): [Khat - Mhat Pi_V[:, :K] | (Kc[:, K:] - Mhat Pi_V[:, K:]) R2];
    //     rows N..2N-1 (Gamma_V): [Pi_V[:, :K] | Pi_V[:, K:] R2]
    for (int e = lane; e < 2 * N * N; e += WAVE) {
        const int r = e / N, c = e % N;
        double v;
        if (r < N) {
            if (c < K) {
                v = (r >= K ? Kc[r * N + c] : 0.0) - A1[r * N + c];
            } else {
                v = 0.0;
                for (int l = 0; l < K; ++l) v = fma(Kc[r * N + K + l] - A1[r * N + K + l], R2[l * K + (c - K)], v);
            }
        } else {
            const int rr = r - N;
            if (c < K) {
                v = PV[rr * N + c];
            } else {
                v = 0.0;
                for (int l = 0; l < K; ++l) v = fma(PV[rr * N + K + l], R2[l * K + (c - K)], v);
            }
        }
        a.out[0][e] = v;
    }
    // S_V rows 0..N-1 (B_V): [Kc[:K, :]^T - Mhat^T Pi_U[:, :K] | [0; Kc[:K, K:]^T] - Mhat^T Pi_U[:, :K] |
    //                         (Kc[K:, :]^T - Mhat^T Pi_U[:, K:]) R1];
    //     rows N..2N-1 (Gamma_U): [Pi_U[:, :K] | Pi_U[:, :K] | Pi_U[:, K:] R1]
    for (int e = lane; e < 2 * N * 3 * K; e += WAVE) {
        const int r = e / (3 * K), c = e % (3 * K);
        double v;
        if (r < N) {
            if (c < K) {
                v = Kc[c * N + r] - A2[r * N + c];
            } else if (c < 2 * K) {
                v = (r >= K ? Kc[(c - K) * N + r] : 0.0) - A2[r * N + (c - K)];
            } else {
                v = 0.0;
                for (int l = 0; l < K; ++l) v = fma(Kc[(K + l) * N + r] - A2[r * N + K + l], R1[l * K + (c - 2 * K)], v);
            }
        } else {
            const int rr = r - N;
            if (c < 2 * K) {
                v = PU[rr * N + (c % K)];
            } else {
                v = 0.0;
                for (int l = 0; l < K; ++l) v = fma(PU[rr * N + K + l], R1[l * K + (c - 2 * K)], v);
            }
        }
        a.out[1][e] = v;
    }
}

// in[0] = U~^T G_U, in[1] = V~^T G_V, in[2] = R_A^{-1}, in[3] = R_B^{-1} ->
// out[0] = [[R_A^{-T}], [-(U~^T G_U) R_A^{-T}]] (2K x K) for Abar = [G_U | U~] S; out[1] likewise
template <int K>
__device__ void tail_abar(const TailArgs& a) {
    const int lane = lane_id();
    for (int side = 0; side < 2; ++side) {
        const double* G = a.in[side];
        const double* Ri = a.in[2 + side];
        for (int e = lane; e < 2 * K * K; e += WAVE) {
            const int r = e / K, c = e % K;
            double v;
            if (r < K) {
                v = Ri[c * K + r];
            } else {
                v = 0.0;
                for (int l = 0; l < K; ++l) v = fma(G[(r - K) * K + l], Ri[c * K + l], v);
                v = -v;
            }
            a.out[side][e] = v;
        }
    }
}

// in[0] = U^T Ubar_trim, in[1] = V^T Vbar_trim, in[2] = sigma ->
// out[0] = [[Sigma^{-1}], [-(U^T Ubar_trim) Sigma^{-1}]] (2K x K) for F1 = [Ubar_trim | U] S; out[1] likewise
template <int K>
__device__ void tail_f(const TailArgs& a) {
    const int lane = lane_id();
    for (int side = 0; side < 2; ++side) {
        const double* G = a.in[side];
        for (int e = lane; e < 2 * K * K; e += WAVE) {
            const int r = e / K, c = e % K;
            const double is = 1.0 / a.in[2][c];
            a.out[side][e] = r < K ? (r == c ? is : 0.0) : -G[(r - K) * K + c] * is;
        }
    }
}

// Gamma for the previous body. in[0] = [U_k | F1 | P]^T B_U' ((2K + rt) x 2K),
// in[1] = [V_k | F2 | Q]^T B_V', in[2] = sigma_k, in[3] = ||P Q^T||^2 (one value).
// out[0] = S for Gamma_V' = [H_V | F1 | U_k | P] S (rows 2K + K + K + rt, 2K columns),
// out[1] = S for Gamma_U' = [H_U | F2 | V_k | Q] S.
// init: the first reverse step: Gamma_V = [U_K | P] S (rows K + rt) from
// in[1] = [V_K | Q]^T B_V; Gamma_U = [V_K | Q] S from in[0] = [U_K | P]^T B_U.
template <int K>
__device__ void tail_gamma(const TailArgs& a) {
    constexpr int N = 2 * K;
    const int lane = lane_id();
    const int rt = a.rt;
    const double c = a.c / a.in[3][0];
    for (int side = 0; side < 2; ++side) {
        // Gamma_V (side 0) takes the V-side Gram, Gamma_U (side 1) the U-side one
        const double* G = a.in[side == 0 ? 1 : 0];
        // G rows: [X_k (K) | F (K) | T (rt)] (init: [X_k (K) | T (rt)])
        const int offT = a.init ? K : 2 * K;
        const int rows = a.init ? K + rt : 2 * N + rt;
        for (int e = lane; e < rows * N; e += WAVE) {
            const int r = e / N, col = e % N;
            double v;
            if (a.init) {
                v = r < K ? c * a.in[2][r] * G[r * N + col] : -c * G[(offT + r - K) * N + col];
            } else if (r < N) {
                v = (r == col) ? 1.0 : 0.0;
            } else if (r < N + K) {
                v = G[(r - N) * N + col];                                   // X_k^T B'
            } else if (r < N + 2 * K) {
                const int t = r - N - K;
                v = G[(K + t) * N + col] + c * a.in[2][t] * G[t * N + col];  // F^T B' + c Sigma X_k^T B'
            } else {
                v = -c * G[(offT + r - N - 2 * K) * N + col];
            }
            a.out[side][e] = v;
        }
    }
}

// in[0] = P^T P, in[1] = Q^T Q (rt x rt) -> out[0][0] = ||P Q^T||_F^2
__device__ void tail_nt(const TailArgs& a) {
    const int lane = lane_id();
    double v = 0.0;
    for (int e = lane; e < a.rt * a.rt; e += WAVE) v = fma(a.in[0][e], a.in[1][e], v);
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, WAVE);
    if (lane == 0) a.out[0][0] = v;
}

// in[0] = U_0^T ((Zbar o s') V_0) (K x K), in[1] = sigma_0 ->
// out[0][t] = sigmabar_t = in[0][t][t]; out[1] = [[Sigma], [I]] (2K x K)
template <int K>
__device__ void tail_out0(const TailArgs& a) {
    const int lane = lane_id();
    if (lane < K) a.out[0][lane] = a.in[0][lane * K + lane];
    for (int e = lane; e < 2 * K * K; e += WAVE) {
        const int r = e / K, c = e % K;
        a.out[1][e] = r < K ? (r == c ? a.in[1][c] : 0.0) : ((r - K) == c ? 1.0 : 0.0);
    }
}

// out[0] = [[I], [I]] (2K x K): the sum of two K-wide panels
template <int K>
__device__ void tail_i2(const TailArgs& a) {
    const int lane = lane_id();
    for (int e = lane; e < 2 * K * K; e += WAVE) a.out[0][e] = ((e / K) % K == e % K) ? 1.0 : 0.0;
}

enum TailMode : int {
    T_CHOL = 0, T_C = 1, T_M = 2, T_B2 = 3, T_ABAR = 4, T_F = 5, T_GAMMA = 6, T_NT = 7, T_OUT0 = 8, T_I2 = 9
};

template <int K>
__global__ __launch_bounds__(WAVE) void k_adj_tail(TailArgs a, int mode) {
    switch (mode) {
        case T_CHOL: tail_chol<K>(a); break;
        case T_C: tail_c<K>(a); break;
        case T_M: tail_m<K>(a); break;
        case T_B2: tail_b2<K>(a); break;
        case T_ABAR: tail_abar<K>(a); break;
        case T_F: tail_f<K>(a); break;
        case T_GAMMA: tail_gamma<K>(a); break;
        case T_NT: tail_nt(a); break;
        case T_OUT0: tail_out0<K>(a); break;
        case T_I2: tail_i2<K>(a); break;
        default: break;
    }
}

__global__ void k_adj_zero(uint32_t* p, int count) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < count) p[i] = 0u;
}

// ---- host side ------------------------------------------------------------------------

inline int nblk_rows(int rows, int per) { return (rows + per - 1) / per; }

PanelRef pr(const double* p, int ld, int w) {
    PanelRef r;
    r.p = p;
    r.ld = ld;
    r.w = w;
    return r;
}

struct Host {
    const AdjointProblem& P;
    const AdjointBufs& B;
    hipStream_t s;
    int K, m, n;

    // small-matrix slot i (AJ_GE doubles each)
    double* sm(int i) const { return B.small + (size_t)i * AJ_GE; }

    hipError_t gram(const PanelRef* Lu, int nLu, const PanelRef* Ru, int nRu, double* outU, const PanelRef* Lv,
                    int nLv, const PanelRef* Rv, int nRv, double* outV) const {
        GramArgs g;
        memset(&g, 0, sizeof(g));
        const PanelRef* Ls[2] = {Lu, Lv};
        const PanelRef* Rs[2] = {Ru, Rv};
        const int nL[2] = {nLu, nLv}, nR[2] = {nRu, nRv};
        double* outs[2] = {outU, outV};
        const int rows[2] = {m, n};
        for (int side = 0; side < 2; ++side) {
            GramJob& J = g.job[side];
            if (!outs[side]) continue;
            J.nL = nL[side];
            J.nR = nR[side];
            for (int q = 0; q < J.nL; ++q) {
                J.L[q] = Ls[side][q];
                J.wL += J.L[q].w;
            }
            for (int q = 0; q < J.nR; ++q) {
                J.R[q] = Rs[side][q];
                J.wR += J.R[q].w;
            }
            if (J.wL + J.wR > AJ_GW || J.wL * J.wR > AJ_GE) return hipErrorInvalidValue;
            J.rows = rows[side];
            J.out = outs[side];
            g.nblk[side] = nblk_rows(rows[side], AJ_ROWS);
        }
        g.gpart = B.gpart;
        g.cnt = B.cnt;
        const int blocks = g.nblk[0] + g.nblk[1];
        if (blocks == 0) return hipSuccess;
        hipLaunchKernelGGL(k_adj_gram, dim3(blocks), dim3(256), 0, s, g);
        return hipGetLastError();
    }

    hipError_t combine(const PanelRef* inU, int nU, const double* SU, int qU, double* outU, int ldU,
                       const PanelRef* inV, int nV, const double* SV, int qV, double* outV, int ldV) const {
        CombArgs c;
        memset(&c, 0, sizeof(c));
        const PanelRef* ins[2] = {inU, inV};
        const int nin[2] = {nU, nV}, q[2] = {qU, qV}, ld[2] = {ldU, ldV};
        const double* S[2] = {SU, SV};
        double* outs[2] = {outU, outV};
        const int rows[2] = {m, n};
        for (int side = 0; side < 2; ++side) {
            if (!outs[side]) continue;
            CombJob& J = c.job[side];
            J.nin = nin[side];
            for (int t = 0; t < J.nin; ++t) {
                J.in[t] = ins[side][t];
                J.win += J.in[t].w;
            }
            if (J.win * q[side] > AJ_GE) return hipErrorInvalidValue;
            J.rows = rows[side];
            J.q = q[side];
            J.S = S[side];
            J.out = outs[side];
            J.ldo = ld[side];
            c.nblk[side] = (int)(((int64_t)rows[side] * q[side] + 255) / 256);
        }
        const int blocks = c.nblk[0] + c.nblk[1];
        if (blocks == 0) return hipSuccess;
        hipLaunchKernelGGL(k_adj_combine, dim3(blocks), dim3(256), 0, s, c);
        return hipGetLastError();
    }

    hipError_t tail(const TailArgs& t, int mode) const {
        switch (K) {
#define RPCA_CASE(KK) \
    case KK: hipLaunchKernelGGL((k_adj_tail<KK>), dim3(1), dim3(WAVE), 0, s, t, mode); break;
            RPCA_CASE(1) RPCA_CASE(2) RPCA_CASE(3) RPCA_CASE(4) RPCA_CASE(5)
            RPCA_CASE(6) RPCA_CASE(7) RPCA_CASE(8) RPCA_CASE(9) RPCA_CASE(10)
#undef RPCA_CASE
            default: return hipErrorInvalidValue;
        }
        return hipGetLastError();
    }

    template <typename T>
    hipError_t stream_t(const AdjStream& a, bool bwd) const {
        const dim3 grid((unsigned)(a.n_ct * a.n_rt)), block(RX_THREADS);
        switch (K) {
#define RPCA_CASE(KK)                                                                                   \
    case KK:                                                                                            \
        if (bwd) hipLaunchKernelGGL((k_adj_stream<T, KK, true>), grid, block, 0, s, a);                \
        else hipLaunchKernelGGL((k_adj_stream<T, KK, false>), grid, block, 0, s, a);                    \
        break;
            RPCA_CASE(1) RPCA_CASE(2) RPCA_CASE(3) RPCA_CASE(4) RPCA_CASE(5)
            RPCA_CASE(6) RPCA_CASE(7) RPCA_CASE(8) RPCA_CASE(9) RPCA_CASE(10)
#undef RPCA_CASE
            default: return hipErrorInvalidValue;
        }
        return hipGetLastError();
    }

    // one pass over D at checkpoint k and its tile sums into SR (m x W) and SC (n x W)
    hipError_t pass(int k, bool bwd, AdjStream a, int W, double* SR, double* SC, double* scal_out) const {
        a.D = P.D;
        a.ldd = P.ldd;
        a.m = m;
        a.n = n;
        a.TM = P.TM;
        a.n_ct = P.n_ct;
        a.n_rt = P.n_rt;
        a.U = P.U[k];
        a.sig = P.sigma[k];
        a.V = P.V[k];
        a.zeta = P.zeta[k];
        a.tau = P.tau[k];
        a.Rp = B.Rp;
        a.Cp = B.Cp;
        a.scal = B.scal;
        hipError_t e = P.dtype == 1 ? stream_t<float>(a, bwd) : stream_t<double>(a, bwd);
        if (e != hipSuccess) return e;
        SumArgs sa;
        sa.Rp = B.Rp;
        sa.Cp = B.Cp;
        sa.scal = B.scal;
        sa.SR = SR;
        sa.SC = SC;
        sa.scal_out = scal_out;
        sa.m = m;
        sa.n = n;
        sa.W = W;
        sa.n_ct = P.n_ct;
        sa.n_rt = P.n_rt;
        const int64_t tot = (int64_t)(m + n) * W;
        hipLaunchKernelGGL(k_adj_sum, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, s, sa);
        return hipGetLastError();
    }

    // Forward recompute of body k into slot sl: trim, bases, Y1/Y2, complements,
    // B_U = [U~ Q1], B_V = [V~ Q2], R1, R2 and the SVD of M.
    hipError_t forward(int k, int sl) const {
        const AdjointBufs::Slot& S = B.slot[sl];
        const int N = 2 * K;
        TrimArgs ta;
        memset(&ta, 0, sizeof(ta));
        ta.X[0] = P.U[k];
        ta.X[1] = P.V[k];
        ta.A[0] = S.Am;
        ta.A[1] = S.Bm;
        ta.w[0] = S.wU;
        ta.w[1] = S.wV;
        ta.rho[0] = S.rhoU;
        ta.rho[1] = S.rhoV;
        ta.c[0] = P.cU;
        ta.c[1] = P.cV;
        ta.rows[0] = m;
        ta.rows[1] = n;
        ta.nblk0 = nblk_rows(m, 256);
        ta.K = K;
        hipLaunchKernelGGL(k_adj_trim, dim3((unsigned)(ta.nblk0 + nblk_rows(n, 256))), dim3(256), 0, s, ta, 0);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
        PanelRef a1[1] = {pr(S.Am, K, K)}, b1[1] = {pr(S.Bm, K, K)};
        if ((e = gram(a1, 1, a1, 1, sm(0), b1, 1, b1, 1, sm(1))) != hipSuccess) return e;
        TailArgs t;
        memset(&t, 0, sizeof(t));
        t.in[0] = sm(0);
        t.in[1] = sm(1);
        t.out[0] = S.RAinv;
        t.out[1] = S.RBinv;
        if ((e = tail(t, T_CHOL)) != hipSuccess) return e;
        // U~ = A R_A^{-1} into the first K columns of B_U (row stride 2K)
        if ((e = combine(a1, 1, S.RAinv, K, S.BU, N, b1, 1, S.RBinv, K, S.BV, N)) != hipSuccess) return e;
        // Y1 = Z V~, Y2 = Z^T U~
        AdjStream a;
        memset(&a, 0, sizeof(a));
        a.ro0 = pr(S.BV, N, K);
        a.co0 = pr(S.BU, N, K);
        a.hw = 0;
        if ((e = pass(k, false, a, K, B.Y1, B.Y2, B.scal_out)) != hipSuccess) return e;
        PanelRef ut[1] = {pr(S.BU, N, K)}, vt[1] = {pr(S.BV, N, K)};
        PanelRef y1[1] = {pr(B.Y1, K, K)}, y2[1] = {pr(B.Y2, K, K)};
        if ((e = gram(ut, 1, y1, 1, sm(2), vt, 1, y2, 1, sm(3))) != hipSuccess) return e;
        memset(&t, 0, sizeof(t));
        t.in[0] = sm(2);
        t.in[1] = sm(3);
        t.out[0] = sm(4);
        t.out[1] = sm(5);
        t.out[2] = S.C;
        if ((e = tail(t, T_C)) != hipSuccess) return e;
        // W1 = Y1 - U~ C, W2 = Y2 - V~ (V~^T Y2)
        PanelRef iw1[2] = {pr(B.Y1, K, K), pr(S.BU, N, K)}, iw2[2] = {pr(B.Y2, K, K), pr(S.BV, N, K)};
        if ((e = combine(iw1, 2, sm(4), K, B.W1, K, iw2, 2, sm(5), K, B.W2, K)) != hipSuccess) return e;
        PanelRef w1[1] = {pr(B.W1, K, K)}, w2[1] = {pr(B.W2, K, K)};
        if ((e = gram(w1, 1, w1, 1, sm(6), w2, 1, w2, 1, sm(7))) != hipSuccess) return e;
        memset(&t, 0, sizeof(t));
        t.in[0] = sm(6);
        t.in[1] = sm(7);
        t.out[0] = S.R1inv;
        t.out[1] = S.R2inv;
        t.out[2] = S.R1;
        t.out[3] = S.R2;
        if ((e = tail(t, T_CHOL)) != hipSuccess) return e;
        memset(&t, 0, sizeof(t));
        t.in[0] = S.C;
        t.in[1] = S.R1;
        t.in[2] = S.R2;
        t.out[0] = S.UM;
        t.out[1] = S.SM;
        t.out[2] = S.VM;
        if ((e = tail(t, T_M)) != hipSuccess) return e;
        // Q1 = W1 R1^{-1} into the last K columns of B_U, Q2 likewise
        PanelRef q1[1] = {pr(B.W1, K, K)}, q2[1] = {pr(B.W2, K, K)};
        return combine(q1, 1, S.R1inv, K, S.BU + K, N, q2, 1, S.R2inv, K, S.BV + K, N);
    }
};

}  // namespace

size_t adjoint_ws_bytes(int64_t m, int64_t n, int K, int n_ct, int n_rt) {
    AdjointBufs b;
    (void)adjoint_carve(reinterpret_cast<void*>(uintptr_t(256)), m, n, K, n_ct, n_rt, &b);
    return (size_t)(b.end - reinterpret_cast<char*>(uintptr_t(256)));
}

hipError_t adjoint_carve(void* base, int64_t m, int64_t n, int K, int n_ct, int n_rt, AdjointBufs* b) {
    char* p = static_cast<char*>(base);
    auto take = [&](size_t count) {
        double* r = reinterpret_cast<double*>(p);
        p += ((count * sizeof(double) + 255) / 256) * 256;
        return r;
    };
    const int N = 2 * K;
    const size_t W = 3 * (size_t)K;
    for (int sl = 0; sl < 2; ++sl) {
        AdjointBufs::Slot& S = b->slot[sl];
        S.Am = take(m * K);
        S.wU = take(m);
        S.rhoU = take(m);
        S.BU = take(m * N);
        S.Bm = take(n * K);
        S.wV = take(n);
        S.rhoV = take(n);
        S.BV = take(n * N);
        S.RAinv = take(AJ_GE);
        S.RBinv = take(AJ_GE);
        S.C = take(AJ_GE);
        S.R1 = take(AJ_GE);
        S.R2 = take(AJ_GE);
        S.R1inv = take(AJ_GE);
        S.R2inv = take(AJ_GE);
        S.UM = take(AJ_GE);
        S.SM = take(AJ_GE);
        S.VM = take(AJ_GE);
    }
    b->Y1 = take(m * K);
    b->W1 = take(m * K);
    b->GammaV = take(m * N);
    b->YG = take(m * N);
    b->SR = take(m * W);
    b->GU = take(m * K);
    b->Abar = take(m * K);
    b->Utrim = take(m * K);
    b->F1 = take(m * K);
    b->Y2 = take(n * K);
    b->W2 = take(n * K);
    b->GammaU = take(n * N);
    b->XG = take(n * 3 * K);
    b->SC = take(n * W);
    b->GV = take(n * K);
    b->Bbar = take(n * K);
    b->Vtrim = take(n * K);
    b->F2 = take(n * K);
    b->Rp = take((size_t)n_ct * m * W);
    b->Cp = take((size_t)n_rt * n * W);
    b->scal = take(2 * (size_t)n_ct * n_rt);
    b->scal_out = take(8);
    const size_t gblk = (size_t)((m + AJ_ROWS - 1) / AJ_ROWS + (n + AJ_ROWS - 1) / AJ_ROWS);
    b->gpart = take(gblk * AJ_GE);
    b->small = take(16 * (size_t)AJ_GE);
    b->zbar = take(RPCA_MAX_UNROLL);
    b->cnt = reinterpret_cast<uint32_t*>(take(32));   // 64 counters
    b->end = p;
    return hipSuccess;
}

hipError_t adjoint_run(const AdjointProblem& P, const AdjointBufs& B, hipStream_t s) {
    Host h{P, B, s, P.K, (int)P.m, (int)P.n};
    const int K = P.K, N = 2 * K, Kt = P.Kt, rt = P.rt;
    hipLaunchKernelGGL(k_adj_zero, dim3(1), dim3(64), 0, s, B.cnt, 64);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    // ||P Q^T||^2
    PanelRef pp[1] = {pr(P.P, rt, rt)}, qq[1] = {pr(P.Q, rt, rt)};
    if ((e = h.gram(pp, 1, pp, 1, h.sm(10), qq, 1, qq, 1, h.sm(11))) != hipSuccess) return e;
    TailArgs t;
    memset(&t, 0, sizeof(t));
    t.in[0] = h.sm(10);
    t.in[1] = h.sm(11);
    t.out[0] = h.sm(12);
    t.rt = rt;
    if ((e = h.tail(t, T_NT)) != hipSuccess) return e;
    double* nt = h.sm(12);
    // body Kt - 1 forward, then Gamma from the loss term of L_Kt
    int sl = (Kt - 1) & 1;
    if ((e = h.forward(Kt - 1, sl)) != hipSuccess) return e;
    {
        const AdjointBufs::Slot& S = B.slot[sl];
        PanelRef lu[2] = {pr(P.U[Kt], K, K), pr(P.P, rt, rt)}, ru[1] = {pr(S.BU, N, N)};
        PanelRef lv[2] = {pr(P.V[Kt], K, K), pr(P.Q, rt, rt)}, rv[1] = {pr(S.BV, N, N)};
        if ((e = h.gram(lu, 2, ru, 1, h.sm(13), lv, 2, rv, 1, h.sm(14))) != hipSuccess) return e;
        memset(&t, 0, sizeof(t));
        t.in[0] = h.sm(13);
        t.in[1] = h.sm(14);
        t.in[2] = P.sigma[Kt];
        t.in[3] = nt;
        t.out[0] = h.sm(4);
        t.out[1] = h.sm(5);
        t.c = 2.0 * P.weight[Kt - 1];
        t.rt = rt;
        t.init = 1;
        if ((e = h.tail(t, T_GAMMA)) != hipSuccess) return e;
        if ((e = h.combine(lu, 2, h.sm(4), N, B.GammaV, N, lv, 2, h.sm(5), N, B.GammaU, N)) != hipSuccess) return e;
    }
    for (int k = Kt - 1; k >= 0; --k) {
        sl = k & 1;
        const AdjointBufs::Slot& S = B.slot[sl];
        const AdjointBufs::Slot& Sp = B.slot[sl ^ 1];
        // H_r: Mhat = B_U^T Gamma_V, then [Y_ | GU0] and [X_ | N_V | GV0]
        PanelRef bu[1] = {pr(S.BU, N, N)}, gv[1] = {pr(B.GammaV, N, N)};
        if ((e = h.gram(bu, 1, gv, 1, h.sm(0), nullptr, 0, nullptr, 0, nullptr)) != hipSuccess) return e;
        memset(&t, 0, sizeof(t));
        t.in[0] = h.sm(0);
        t.in[1] = S.UM;
        t.in[2] = S.SM;
        t.in[3] = S.VM;
        t.in[4] = S.R1;
        t.in[5] = S.R2;
        t.out[0] = h.sm(1);
        t.out[1] = h.sm(2);
        if ((e = h.tail(t, T_B2)) != hipSuccess) return e;
        PanelRef iu[2] = {pr(S.BU, N, N), pr(B.GammaV, N, N)}, iv[2] = {pr(S.BV, N, N), pr(B.GammaU, N, N)};
        if ((e = h.combine(iu, 2, h.sm(1), N, B.YG, N, iv, 2, h.sm(2), 3 * K, B.XG, 3 * K)) != hipSuccess) return e;
        // the previous body's bases (its forward recompute) for the Hadamard products
        if (k >= 1 && (e = h.forward(k - 1, sl ^ 1)) != hipSuccess) return e;
        // pass over D at L_k: Z N_V | h B_V', Z^T N_U | h B_U', dloss/dzeta_k
        AdjStream a;
        memset(&a, 0, sizeof(a));
        a.ro0 = pr(B.XG + K, 3 * K, K);         // N_V
        a.co0 = pr(B.YG, N, K);                 // N_U = Y_
        if (k >= 1) {
            a.hw = N;
            a.ro1 = pr(Sp.BV, N, N);
            a.co1 = pr(Sp.BU, N, N);
        } else {
            a.hw = K;
            a.ro1 = pr(P.V[0], K, K);
            a.co1 = pr(P.U[0], K, K);
        }
        a.Uz = pr(S.BU, N, K);
        a.Vz = pr(S.BV, N, K);
        a.Xz = pr(B.XG, 3 * K, K);
        a.Yz = pr(B.YG, N, K);
        const int W = K + a.hw;
        if ((e = h.pass(k, true, a, W, B.SR, B.SC, B.scal_out + 2 * 0)) != hipSuccess) return e;
        if ((e = hipMemcpyAsync(P.zeta_bar_dev + k, B.scal_out + 1, sizeof(double), hipMemcpyDeviceToDevice, s)) !=
            hipSuccess)
            return e;
        // G_U = GU0 + Z N_V, G_V = GV0 + Z^T N_U
        double* I2 = h.sm(3);
        {
            TailArgs ti;
            memset(&ti, 0, sizeof(ti));
            ti.out[0] = I2;
            if ((e = h.tail(ti, T_I2)) != hipSuccess) return e;
        }
        PanelRef gu_in[2] = {pr(B.YG + K, N, K), pr(B.SR, W, K)};
        PanelRef gv_in[2] = {pr(B.XG + 2 * K, 3 * K, K), pr(B.SC, W, K)};
        if ((e = h.combine(gu_in, 2, I2, K, B.GU, K, gv_in, 2, I2, K, B.GV, K)) != hipSuccess) return e;
        // Abar = (G_U - U~ (U~^T G_U)) R_A^{-T}, Bbar likewise
        PanelRef ut[1] = {pr(S.BU, N, K)}, vt[1] = {pr(S.BV, N, K)};
        PanelRef gu[1] = {pr(B.GU, K, K)}, gvv[1] = {pr(B.GV, K, K)};
        if ((e = h.gram(ut, 1, gu, 1, h.sm(6), vt, 1, gvv, 1, h.sm(7))) != hipSuccess) return e;
        memset(&t, 0, sizeof(t));
        t.in[0] = h.sm(6);
        t.in[1] = h.sm(7);
        t.in[2] = S.RAinv;
        t.in[3] = S.RBinv;
        t.out[0] = h.sm(8);
        t.out[1] = h.sm(9);
        if ((e = h.tail(t, T_ABAR)) != hipSuccess) return e;
        PanelRef ia[2] = {pr(B.GU, K, K), pr(S.BU, N, K)}, ib[2] = {pr(B.GV, K, K), pr(S.BV, N, K)};
        if ((e = h.combine(ia, 2, h.sm(8), K, B.Abar, K, ib, 2, h.sm(9), K, B.Bbar, K)) != hipSuccess) return e;
        // Trim, reversed
        TrimArgs ta;
        memset(&ta, 0, sizeof(ta));
        ta.X[0] = P.U[k];
        ta.X[1] = P.V[k];
        ta.Abar[0] = B.Abar;
        ta.Abar[1] = B.Bbar;
        ta.Xbar[0] = B.Utrim;
        ta.Xbar[1] = B.Vtrim;
        ta.c[0] = P.cU;
        ta.c[1] = P.cV;
        ta.rows[0] = (int)P.m;
        ta.rows[1] = (int)P.n;
        ta.nblk0 = nblk_rows((int)P.m, 256);
        ta.K = K;
        hipLaunchKernelGGL(k_adj_trim, dim3((unsigned)(ta.nblk0 + nblk_rows((int)P.n, 256))), dim3(256), 0, s, ta, 1);
        if ((e = hipGetLastError()) != hipSuccess) return e;
        if (k == 0) {
            // gradients of the free factors of L_0
            PanelRef u0[1] = {pr(P.U[0], K, K)}, hv0[1] = {pr(B.SR + K, W, K)};
            if ((e = h.gram(u0, 1, hv0, 1, h.sm(6), nullptr, 0, nullptr, 0, nullptr)) != hipSuccess) return e;
            memset(&t, 0, sizeof(t));
            t.in[0] = h.sm(6);
            t.in[1] = P.sigma[0];
            t.out[0] = P.sigma_bar;
            t.out[1] = h.sm(7);
            if ((e = h.tail(t, T_OUT0)) != hipSuccess) return e;
            PanelRef ou[2] = {pr(B.SR + K, W, K), pr(B.Utrim, K, K)};
            PanelRef ov[2] = {pr(B.SC + K, W, K), pr(B.Vtrim, K, K)};
            if ((e = h.combine(ou, 2, h.sm(7), K, P.U_bar, K, ov, 2, h.sm(7), K, P.V_bar, K)) != hipSuccess) return e;
            break;
        }
        // to L_k: F1 = (I - U U^T) Ubar_trim Sigma^{-1}, F2 likewise
        PanelRef uk[1] = {pr(P.U[k], K, K)}, vk[1] = {pr(P.V[k], K, K)};
        PanelRef utr[1] = {pr(B.Utrim, K, K)}, vtr[1] = {pr(B.Vtrim, K, K)};
        if ((e = h.gram(uk, 1, utr, 1, h.sm(6), vk, 1, vtr, 1, h.sm(7))) != hipSuccess) return e;
        memset(&t, 0, sizeof(t));
        t.in[0] = h.sm(6);
        t.in[1] = h.sm(7);
        t.in[2] = P.sigma[k];
        t.out[0] = h.sm(8);
        t.out[1] = h.sm(9);
        if ((e = h.tail(t, T_F)) != hipSuccess) return e;
        PanelRef if1[2] = {pr(B.Utrim, K, K), pr(P.U[k], K, K)}, if2[2] = {pr(B.Vtrim, K, K), pr(P.V[k], K, K)};
        if ((e = h.combine(if1, 2, h.sm(8), K, B.F1, K, if2, 2, h.sm(9), K, B.F2, K)) != hipSuccess) return e;
        // Gamma for body k - 1: Lbar_k = Zbar o s'(X_k) + F1 V^T + U F2^T + c_k (L_k - P Q^T)
        PanelRef lu[3] = {pr(P.U[k], K, K), pr(B.F1, K, K), pr(P.P, rt, rt)}, ru[1] = {pr(Sp.BU, N, N)};
        PanelRef lv[3] = {pr(P.V[k], K, K), pr(B.F2, K, K), pr(P.Q, rt, rt)}, rv[1] = {pr(Sp.BV, N, N)};
        if ((e = h.gram(lu, 3, ru, 1, h.sm(13), lv, 3, rv, 1, h.sm(14))) != hipSuccess) return e;
        memset(&t, 0, sizeof(t));
        t.in[0] = h.sm(13);
        t.in[1] = h.sm(14);
        t.in[2] = P.sigma[k];
        t.in[3] = nt;
        t.out[0] = h.sm(4);
        t.out[1] = h.sm(5);
        t.c = 2.0 * P.weight[k - 1];
        t.rt = rt;
        t.init = 0;
        if ((e = h.tail(t, T_GAMMA)) != hipSuccess) return e;
        PanelRef gvi[4] = {pr(B.SR + K, W, N), pr(B.F1, K, K), pr(P.U[k], K, K), pr(P.P, rt, rt)};
        PanelRef gui[4] = {pr(B.SC + K, W, N), pr(B.F2, K, K), pr(P.V[k], K, K), pr(P.Q, rt, rt)};
        if ((e = h.combine(gvi, 4, h.sm(4), N, B.GammaV, N, gui, 4, h.sm(5), N, B.GammaU, N)) != hipSuccess) return e;
    }
    return hipSuccess;
}

}  // namespace rpca
