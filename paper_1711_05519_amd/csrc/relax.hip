// One AccAltProj iteration with a relaxed threshold and the derivative of a
// loss of the next iterate with respect to the threshold (training of a
// learned threshold schedule; not part of the paper).
//
// From L_k = U diag(sigma) V^T, with x = D - L_k and the relaxation
//   s(x) = x * logistic((|x| - zeta) / tau)       (T_zeta as tau -> 0)
// the iteration forms Z = D - s(x), P_T(Z) on the tangent space of Trim(L_k)
// (Section 2.1) and L_{k+1} = H_r(P_T(Z)). Its derivative in zeta is
//   dZ = dZ/dzeta = x * g (1 - g) / tau,  g = logistic((|x| - zeta) / tau),
// P_T is linear, and H_r moves by its first-order perturbation. Both P_T(Z)
// and P_T(dZ) lie in span[U*, W1, dW1] x span[V*, W2, dW2] (W, dW the
// complements of Z V* and dZ V*), a 3r x 3r reduced space with orthonormal
// bases B_U, B_V, so
//   L_{k+1} = B_U H_r(M) B_V^T,   dL_{k+1} = B_U U_M F V_M^T B_V^T
// with M, dM the 3r x 3r reductions, M = U_M S V_M^T, E = U_M^T dM V_M and
//   F_ij = E_ij (i, j < r);  F_ij = (s_i^2 E_ij + s_i s_j E_ji) / (s_i^2 - s_j^2),
//   F_ji = (s_i^2 E_ji + s_i s_j E_ij) / (s_i^2 - s_j^2)  (i < r <= j);  0 else.
// The loss is ||L_{k+1} - P Q^T||_F^2 / ||P Q^T||_F^2 for given factors P, Q
// (the ground truth of a synthetic instance); it and its derivative need only
// projections of P and Q onto B_U and B_V.
//
// Kernels: one pass over D giving [Y1 dY1] = [Z dZ] V_f and [Y2 dY2] = [Z dZ]^T U_f
// as per-tile partials (plus the relaxed residual); their sums; the products
// [U_f | Y1 dY1 | P]^T [...] (for C, dC and U*^T P); the explicit complements
// [W1 dW1] = [Y1 dY1] R_V^{-1} - U* [C dC] (and the V side), formed row by row
// in FP64 as the FP64 loop path does (Gram differences would cancel); their
// exact Grams with the target factors; a single-wave FP64 tail with the
// small algebra; and the row update of the new factors.

#include "launch.hpp"
#include "wave.hpp"

namespace rpca {
namespace {

template <typename T> __device__ inline const T* cptr(const void* p) { return static_cast<const T*>(p); }

__device__ inline double logistic(double u) { return 0.5 * (1.0 + tanh(0.5 * u)); }

// ---- the pass over D -----------------------------------------------------------
//
// Tile RX_TM x 256: one thread per column; per row the 2K row products are
// summed over the workgroup (wave shuffles, then LDS in wave order).
template <typename T, int K>
__global__ __launch_bounds__(RX_THREADS) void k_relax_stream(RelaxArgs a) {
    constexpr int K2 = 2 * K;
    const T* __restrict__ D = cptr<T>(a.D);
    const T* __restrict__ AL = cptr<T>(a.AL);
    const T* __restrict__ BL = cptr<T>(a.BL);
    const T* __restrict__ Uf = cptr<T>(a.Uf);
    const T* __restrict__ Vf = cptr<T>(a.Vf);
    const int lane = threadIdx.x & (WAVE - 1), wave = threadIdx.x / WAVE;
    const int ct = blockIdx.x % a.n_ct, rt = blockIdx.x / a.n_ct;
    const int j = ct * RX_THREADS + threadIdx.x;
    const bool valid = j < a.n;
    const int i_lo = rt * a.TM, i_hi = min(a.m, i_lo + a.TM);
    const double zeta = a.zeta, tau = a.tau;
    double bl[K], vt[K], y2[K2];
#pragma unroll
    for (int t = 0; t < K; ++t) {
        bl[t] = valid ? static_cast<double>(BL[(size_t)j * K + t]) : 0.0;
        vt[t] = valid ? static_cast<double>(Vf[(size_t)j * K + t]) : 0.0;
    }
#pragma unroll
    for (int t = 0; t < K2; ++t) y2[t] = 0.0;
    __shared__ double red[RX_THREADS / WAVE][K2];
    __shared__ double bred[RX_THREADS / WAVE];
    double res = 0.0;
    for (int i = i_lo; i < i_hi; ++i) {
        double p[K2];
        double x = valid ? static_cast<double>(D[(size_t)i * a.ldd + j]) : 0.0;
        const double d = x;
#pragma unroll
        for (int t = 0; t < K; ++t) x -= static_cast<double>(AL[(size_t)i * K + t]) * bl[t];
        double z = 0.0, zd = 0.0;
        if (valid) {
            const double g = logistic((fabs(x) - zeta) / tau);
            const double s = x * g;
            z = d - s;
            zd = x * g * (1.0 - g) / tau;   // dZ/dzeta = -ds/dzeta
            const double e = x - s;
            res = fma(e, e, res);
        }
#pragma unroll
        for (int t = 0; t < K; ++t) {
            const double u = static_cast<double>(Uf[(size_t)i * K + t]);
            y2[t] = fma(z, u, y2[t]);
            y2[K + t] = fma(zd, u, y2[K + t]);
            p[t] = z * vt[t];
            p[K + t] = zd * vt[t];
        }
#pragma unroll
        for (int t = 0; t < K2; ++t) {
            double v = p[t];
            for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, WAVE);
            p[t] = v;
        }
        if (lane == 0) {
#pragma unroll
            for (int t = 0; t < K2; ++t) red[wave][t] = p[t];
        }
        __syncthreads();
        if (threadIdx.x < K2) {
            double v = 0.0;
            for (int w = 0; w < RX_THREADS / WAVE; ++w) v += red[w][threadIdx.x];
            a.R1[((size_t)ct * a.m + i) * K2 + threadIdx.x] = v;
        }
        __syncthreads();
    }
    if (valid) {
#pragma unroll
        for (int t = 0; t < K2; ++t) a.R2[((size_t)rt * a.n + j) * K2 + t] = y2[t];
    }
    const double tot = block_sum(res, bred);
    if (threadIdx.x == 0) a.Rres[blockIdx.x] = tot;
}

// ---- sums over the tiles --------------------------------------------------------
template <int K>
__global__ __launch_bounds__(256) void k_relax_sum(RelaxArgs a) {
    constexpr int K2 = 2 * K;
    const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
    const int64_t mU = (int64_t)a.m * K2, mV = (int64_t)a.n * K2;
    if (e < mU) {
        double v = 0.0;
        for (int c = 0; c < a.n_ct; ++c) v += a.R1[(size_t)c * mU + e];
        a.RY1[e] = v;
    } else if (e < mU + mV) {
        const int64_t f = e - mU;
        double v = 0.0;
        for (int r = 0; r < a.n_rt; ++r) v += a.R2[(size_t)r * mV + f];
        a.RY2[f] = v;
    }
}

// ---- Grams of [F | Y | P] (WITH_F) or [Y | P] over the rows of each side ----------
//
// The first gU workgroups take rows of the U side (F = U_f, Y = the 2K-wide
// panel RY1, P), the next gV rows of the V side (V_f, RY2, Q). Each writes the
// W x W partial Gram of its 256 rows; the last workgroup sums them in order
// into gram (U side) and gram + RX_WMAX^2 (V side), upper and lower halves.
template <typename T, int K, bool WITH_F>
__global__ __launch_bounds__(256) void k_relax_gram(RelaxArgs a, int cnt_slot, double* gram) {
    constexpr int K2 = 2 * K;
    constexpr int NF = WITH_F ? K : 0;
    const int W = NF + K2 + a.rt_true;
    const bool uside = (int)blockIdx.x < a.gU;
    const int row = (uside ? blockIdx.x : blockIdx.x - a.gU) * 256 + threadIdx.x;
    const int nrows = uside ? a.m : a.n;
    const T* F = cptr<T>(uside ? a.Uf : a.Vf);
    const double* Y = uside ? a.RY1 : a.RY2;
    const double* P = uside ? a.P : a.Q;
    __shared__ double rows[256][RX_WMAX + 1];
    for (int c = 0; c < W; ++c) {
        double v = 0.0;
        if (row < nrows) {
            if (c < NF) v = static_cast<double>(F[(size_t)row * K + c]);
            else if (c < NF + K2) v = Y[(size_t)row * K2 + (c - NF)];
            else v = P[(size_t)row * a.rt_true + (c - NF - K2)];
        }
        rows[threadIdx.x][c] = v;
    }
    __syncthreads();
    double* gp = a.gpartR + (size_t)blockIdx.x * RX_WMAX * RX_WMAX;
    for (int e = threadIdx.x; e < W * W; e += 256) {
        const int p = e / W, q = e % W;
        double v = 0.0;
        if (p <= q)
            for (int r = 0; r < 256; ++r) v = fma(rows[r][p], rows[r][q], v);
        gp[p * RX_WMAX + q] = v;
    }
    __shared__ int flag;
    if (!last_block_arrives(&a.ctrl->cnt[cnt_slot], &flag)) return;
    for (int e = threadIdx.x; e < 2 * W * W; e += 256) {
        const int side = e / (W * W), pq = e % (W * W);
        const int p = pq / W, q = pq % W;
        const int first = side ? a.gU : 0, count = side ? a.gV : a.gU;
        const int lo = p <= q ? p : q, hi = p <= q ? q : p;
        double v = 0.0;
        for (int b = 0; b < count; ++b) v += a.gpartR[(size_t)(first + b) * RX_WMAX * RX_WMAX + lo * RX_WMAX + hi];
        gram[(size_t)side * RX_WMAX * RX_WMAX + p * RX_WMAX + q] = v;
    }
    if (threadIdx.x == 0) a.ctrl->cnt[cnt_slot] = 0;
}

// C = Ra^T (F^T Y_a) Rb and dC = Ra^T (F^T Y_b) Rb from the first Gram
// (F columns 0..K-1, Y columns K..3K-1), lane- or thread-parallel over entries.
template <int K>
__device__ inline void relax_c(const double* G, const double* Ra, const double* Rb, double* Cc, double* Cd,
                               double* tmp, int tid, int nth) {
    for (int e = tid; e < 2 * K * K; e += nth) {
        const int w = e / (K * K), i = (e / K) % K, j = e % K;
        double v = 0.0;
        for (int l = 0; l < K; ++l) v = fma(G[i * RX_WMAX + K + w * K + l], Rb[l * K + j], v);
        tmp[e] = v;   // (F^T Y_w Rb)[i][j]
    }
    __syncthreads();
    for (int e = tid; e < 2 * K * K; e += nth) {
        const int w = e / (K * K), i = (e / K) % K, j = e % K;
        double v = 0.0;
        for (int l = 0; l < K; ++l) v = fma(Ra[l * K + i], tmp[w * K * K + l * K + j], v);
        (w ? Cd : Cc)[i * K + j] = v;
    }
    __syncthreads();
}

// ---- explicit complements, in place of the 2K-wide panels -----------------------
// U side: [W1 dW1] = [Y1 dY1] R_V^{-1} - (U_f R_U^{-1}) [C dC]
// V side: [W2 dW2] = [Y2 dY2] R_U^{-1} - (V_f R_V^{-1}) [C2 dC2]
template <typename T, int K>
__global__ __launch_bounds__(256) void k_relax_complement(RelaxArgs a) {
    constexpr int K2 = 2 * K;
    const bool uside = (int)blockIdx.x < a.gU;
    const int row = (uside ? blockIdx.x : blockIdx.x - a.gU) * 256 + threadIdx.x;
    const int nrows = uside ? a.m : a.n;
    __shared__ double ra[K * K], rb[K * K], cc[K * K], cd[K * K], tmp[2 * K * K];
    const double* RA = uside ? a.RUinv : a.RVinv;   // basis side
    const double* RB = uside ? a.RVinv : a.RUinv;   // product side
    for (int e = threadIdx.x; e < K * K; e += 256) {
        ra[e] = RA[(e / K) * KMAX + e % K];
        rb[e] = RB[(e / K) * KMAX + e % K];
    }
    __syncthreads();
    relax_c<K>(a.gram + (uside ? 0 : RX_WMAX * RX_WMAX), ra, rb, cc, cd, tmp, threadIdx.x, 256);
    if (row >= nrows) return;
    const T* F = cptr<T>(uside ? a.Uf : a.Vf);
    double* Y = uside ? a.RY1 : a.RY2;
    double f[K], fs[K], y[K2];
#pragma unroll
    for (int t = 0; t < K; ++t) f[t] = static_cast<double>(F[(size_t)row * K + t]);
#pragma unroll
    for (int t = 0; t < K2; ++t) y[t] = Y[(size_t)row * K2 + t];
#pragma unroll
    for (int t = 0; t < K; ++t) {
        double v = 0.0;
#pragma unroll
        for (int l = 0; l < K; ++l) v = fma(f[l], ra[l * K + t], v);
        fs[t] = v;   // row of U* (or V*)
    }
#pragma unroll
    for (int t = 0; t < K; ++t) {
        double w = 0.0, wd = 0.0;
#pragma unroll
        for (int l = 0; l < K; ++l) {
            w = fma(y[l], rb[l * K + t], w);
            wd = fma(y[K + l], rb[l * K + t], wd);
            w = fma(-fs[l], cc[l * K + t], w);
            wd = fma(-fs[l], cd[l * K + t], wd);
        }
        Y[(size_t)row * K2 + t] = w;
        Y[(size_t)row * K2 + K + t] = wd;
    }
}

// ---- the small FP64 algebra, one wave ---------------------------------------------

template <int K>
__global__ __launch_bounds__(WAVE) void k_relax_tail(RelaxArgs a) {
    constexpr int K2 = 2 * K, K3 = 3 * K, N = (K3 + 1) / 2 * 2;
    const int lane = lane_id();
    const int rT = a.rt_true;
    constexpr int LD = RX_WMAX;
    // first Grams: [F | Y dY | P]; second: [W dW | P] (U side, then V side)
    const double* G1u = a.gram;
    const double* G1v = a.gram + LD * LD;
    const double* G2u = a.gram2;
    const double* G2v = a.gram2 + LD * LD;
    __shared__ double ru[K * K], rv[K * K], tmp[2 * K * K], t1[K2 * RX_TRUE_MAX];
    __shared__ double C[K * K], Cd[K * K], C2[K * K], C2d[K * K];
    __shared__ double GG[K2 * K2], HH[K2 * K2], RG[K2 * K2], RGi[K2 * K2], RH[K2 * K2], RHi[K2 * K2];
    __shared__ double Ma[N * N], Md[N * N], Mv[N * N], Um[N * N], Vm[N * N], sg[N], Ee[N * N], Fm[N * N];
    __shared__ double Pr[K3 * RX_TRUE_MAX], Qr[K3 * RX_TRUE_MAX];
    __shared__ double PQ[K3 * K3], Hm[K3 * K3], Hd[K3 * K3];
    __shared__ double Z2[K2 * K], out6[6 * K * K];
    for (int e = lane; e < K * K; e += WAVE) {
        ru[e] = a.RUinv[(e / K) * KMAX + e % K];
        rv[e] = a.RVinv[(e / K) * KMAX + e % K];
    }
    wave_sync();
    relax_c<K>(G1u, ru, rv, C, Cd, tmp, lane, WAVE);
    relax_c<K>(G1v, rv, ru, C2, C2d, tmp, lane, WAVE);
    for (int e = lane; e < K2 * K2; e += WAVE) {
        GG[e] = G2u[(e / K2) * LD + e % K2];
        HH[e] = G2v[(e / K2) * LD + e % K2];
    }
    wave_sync();
    w_chol_inv2<K2>(GG, RG, RGi, HH, RH, RHi);
    // reduced M and dM (column-major, N x N, zero padded)
    for (int e = lane; e < N * N; e += WAVE) {
        const int col = e / N, row = e % N;
        double m0 = 0.0, m1 = 0.0;
        if (row < K && col < K) {
            m0 = C[row * K + col];
            m1 = Cd[row * K + col];
        } else if (row < K && col < K3) {
            m0 = RH[(col - K) * K2 + row];
            m1 = RH[(col - K) * K2 + K + row];
        } else if (row < K3 && col < K) {
            m0 = RG[(row - K) * K2 + col];
            m1 = RG[(row - K) * K2 + K + col];
        }
        Ma[e] = m0;
        Md[e] = m1;
    }
    wave_sync();
    const int sweeps = wave_jacobi_svd<N, false>(Ma, Mv, sg, Um, Vm);   // Um, Vm column-major
    // M has rank <= 2K: singular values at the rounding level are zero, and
    // their left vectors (undefined in the one-sided method) are dropped; the
    // left null space then enters through the projector term below.
    {
        const double cut = 1e-12 * sg[0];
        for (int e = lane; e < N * N; e += WAVE)
            if (sg[e / N] <= cut) Um[e] = 0.0;
        wave_sync();
        if (lane < N && sg[lane] <= cut) sg[lane] = 0.0;
        wave_sync();
    }
    // E = U_M^T dM V_M (row-major N x N); dM column-major: element (r, c) = Md[c * N + r]
    for (int e = lane; e < N * N; e += WAVE) {
        const int i = e / N, j = e % N;
        double v = 0.0;
        for (int r = 0; r < N; ++r) {
            double w = 0.0;
            for (int c = 0; c < N; ++c) w = fma(Md[c * N + r], Vm[j * N + c], w);
            v = fma(Um[i * N + r], w, v);
        }
        Ee[e] = v;
    }
    wave_sync();
    for (int e = lane; e < N * N; e += WAVE) {
        const int i = e / N, j = e % N;
        double f = 0.0;
        if (i < K && j < K) {
            f = Ee[e];
        } else if (i < K && j >= K) {
            const double si = sg[i], sj = sg[j];
            f = (si * si * Ee[i * N + j] + si * sj * Ee[j * N + i]) / (si * si - sj * sj);
        } else if (j < K && i >= K) {
            const double si = sg[j], sj = sg[i];
            f = (si * si * Ee[i * N + j] + si * sj * Ee[j * N + i]) / (si * si - sj * sj);
        }
        Fm[e] = f;
    }
    wave_sync();
    // H = U_M[:, :K] S_K V_M[:, :K]^T and dH = U_M F V_M^T on the leading K3 x K3 block
    for (int e = lane; e < K3 * K3; e += WAVE) {
        const int r = e / K3, c = e % K3;
        double h = 0.0, hd = 0.0;
        for (int t = 0; t < K; ++t) h = fma(Um[t * N + r] * sg[t], Vm[t * N + c], h);
        for (int i = 0; i < N; ++i) {
            double w = 0.0;
            for (int j = 0; j < N; ++j) w = fma(Fm[i * N + j], Vm[j * N + c], w);
            hd = fma(Um[i * N + r], w, hd);
        }
        Hm[e] = h;
        Hd[e] = hd;
    }
    wave_sync();
    // left-null-space part of the perturbation: (I - U_M U_M^T) dM V_K V_K^T
    // (in the formula it is the block j >= rank, i < K, with F_ji = E_ji)
    {
        double* Tm = Ee;   // N x K, reuses Ee
        for (int e = lane; e < N * K; e += WAVE) {
            const int r = e / K, t = e % K;
            double v = 0.0;
            for (int c = 0; c < N; ++c) v = fma(Md[c * N + r], Vm[t * N + c], v);
            Tm[e] = v;
        }
        wave_sync();
        double* Pt = Fm;   // N x K, reuses Fm
        for (int e = lane; e < N * K; e += WAVE) {
            const int j = e / K, t = e % K;   // (U_M^T T)[j][t]
            double v = 0.0;
            for (int r = 0; r < N; ++r) v = fma(Um[j * N + r], Tm[r * K + t], v);
            Pt[e] = v;
        }
        wave_sync();
        for (int e = lane; e < N * K; e += WAVE) {
            const int r = e / K, t = e % K;
            double v = Tm[e];
            for (int j = 0; j < N; ++j) v -= Um[j * N + r] * Pt[j * K + t];
            Md[e] = v;   // (I - U U^T) T, N x K, reuses Md
        }
        wave_sync();
        for (int e = lane; e < K3 * K3; e += WAVE) {
            const int r = e / K3, c = e % K3;
            double v = 0.0;
            for (int t = 0; t < K; ++t) v = fma(Md[r * K + t], Vm[t * N + c], v);
            Hd[e] += v;
        }
        wave_sync();
    }
    // projections of the target factors onto the reduced bases:
    // B_U^T P = [R_U^{-T} (U_f^T P) ; R_G^{-T} ([W1 dW1]^T P)], likewise B_V^T Q
    for (int side = 0; side < 2; ++side) {
        const double* G1 = side ? G1v : G1u;
        const double* G2 = side ? G2v : G2u;
        const double* Ra = side ? rv : ru;
        const double* Ri = side ? RHi : RGi;
        double* Out = side ? Qr : Pr;
        for (int e = lane; e < K * rT; e += WAVE) {
            const int i = e / rT, q = e % rT;
            double v = 0.0;
            for (int l = 0; l < K; ++l) v = fma(Ra[l * K + i], G1[l * LD + K3 + q], v);
            Out[e] = v;
        }
        for (int e = lane; e < K2 * rT; e += WAVE) t1[e] = G2[(e / rT) * LD + K2 + e % rT];
        wave_sync();
        for (int e = lane; e < K2 * rT; e += WAVE) {
            const int i = e / rT, q = e % rT;
            double v = 0.0;
            for (int l = 0; l < K2; ++l) v = fma(Ri[l * K2 + i], t1[l * rT + q], v);
            Out[K * rT + e] = v;
        }
        wave_sync();
    }
    for (int e = lane; e < K3 * K3; e += WAVE) {
        const int i = e / K3, j = e % K3;
        double v = 0.0;
        for (int q = 0; q < rT; ++q) v = fma(Pr[i * rT + q], Qr[j * rT + q], v);
        PQ[e] = v;
    }
    wave_sync();
    // ||P Q^T||^2 = tr((P^T P)(Q^T Q)) and the inner products of the loss
    double acc = 0.0, h2 = 0.0, hpq = 0.0, hdh = 0.0, hdpq = 0.0;
    for (int e = lane; e < rT * rT; e += WAVE)
        acc += G2u[(K2 + e / rT) * LD + K2 + e % rT] * G2v[(K2 + e / rT) * LD + K2 + e % rT];
    for (int e = lane; e < K3 * K3; e += WAVE) {
        h2 = fma(Hm[e], Hm[e], h2);
        hpq = fma(Hm[e], PQ[e], hpq);
        hdh = fma(Hm[e], Hd[e], hdh);
        hdpq = fma(Hd[e], PQ[e], hdpq);
    }
    for (int off = 32; off > 0; off >>= 1) {
        acc += __shfl_xor(acc, off, WAVE);
        h2 += __shfl_xor(h2, off, WAVE);
        hpq += __shfl_xor(hpq, off, WAVE);
        hdh += __shfl_xor(hdh, off, WAVE);
        hdpq += __shfl_xor(hdpq, off, WAVE);
    }
    // new factors: U' = [U* Q] U_M[:, :K] = U_f (R_U^{-1} X1) + [W1 dW1] (R_G^{-1} X2)
    for (int side = 0; side < 2; ++side) {
        const double* Xm = side ? Vm : Um;
        const double* Ri = side ? RHi : RGi;
        const double* Ra = side ? rv : ru;
        double* o = out6 + side * 3 * K * K;
        for (int e = lane; e < K2 * K; e += WAVE) {
            const int i = e / K, t = e % K;
            double v = 0.0;
            for (int l = 0; l < K2; ++l) v = fma(Ri[i * K2 + l], Xm[t * N + K + l], v);
            Z2[e] = v;
        }
        for (int e = lane; e < K * K; e += WAVE) {
            const int i = e / K, t = e % K;
            double v = 0.0;
            for (int l = 0; l < K; ++l) v = fma(Ra[i * K + l], Xm[t * N + l], v);
            o[e] = v;
        }
        wave_sync();
        for (int e = lane; e < K2 * K; e += WAVE) o[K * K + e] = Z2[e];
        wave_sync();
    }
    for (int e = lane; e < 6 * K * K; e += WAVE) a.coef[e] = out6[e];
    if (lane < K) a.sigma_out[lane] = sg[lane];
    if (lane == 0) {
        double rs = 0.0;
        for (int b = 0; b < a.n_tiles; ++b) rs += a.Rres[b];
        RelaxResult r;
        r.loss = (h2 - 2.0 * hpq + acc) / acc;
        r.dloss_dzeta = 2.0 * (hdh - hdpq) / acc;
        r.err = sqrt(rs / a.normD2);
        r.sigma1 = sg[0];
        r.sigma_r1 = sg[K];
        r.sweeps = sweeps;
        r.pad = 0;
        *a.result = r;
    }
}

// ---- row update of the new factors: U' = U_f E_F + [W1 dW1] [Za; Zb] ---------------
template <typename T, int K>
__global__ __launch_bounds__(256) void k_relax_update(RelaxArgs a) {
    constexpr int K2 = 2 * K;
    const bool uside = (int)blockIdx.x < a.gU;
    const int row = (uside ? blockIdx.x : blockIdx.x - a.gU) * 256 + threadIdx.x;
    const int nrows = uside ? a.m : a.n;
    __shared__ double cf[3 * K * K];
    for (int e = threadIdx.x; e < 3 * K * K; e += 256) cf[e] = a.coef[(uside ? 0 : 3 * K * K) + e];
    __syncthreads();
    if (row >= nrows) return;
    const T* F = cptr<T>(uside ? a.Uf : a.Vf);
    const double* Y = uside ? a.RY1 : a.RY2;
    double f[K], y[K2];
#pragma unroll
    for (int t = 0; t < K; ++t) f[t] = static_cast<double>(F[(size_t)row * K + t]);
#pragma unroll
    for (int t = 0; t < K2; ++t) y[t] = Y[(size_t)row * K2 + t];
    double* out = uside ? a.Uout : a.Vout;
#pragma unroll
    for (int t = 0; t < K; ++t) {
        double v = 0.0;
#pragma unroll
        for (int l = 0; l < K; ++l) {
            v = fma(f[l], cf[l * K + t], v);
            v = fma(y[l], cf[K * K + l * K + t], v);
            v = fma(y[K + l], cf[2 * K * K + l * K + t], v);
        }
        out[(size_t)row * K + t] = v;
    }
}

template <typename T>
hipError_t relax_dispatch(const RelaxArgs& a, hipStream_t s) {
    const unsigned gs = (unsigned)(a.n_ct * a.n_rt);
    const unsigned gsum = (unsigned)((((int64_t)a.m + a.n) * 2 * a.K + 255) / 256);
    const unsigned gpan = (unsigned)(a.gU + a.gV);
    switch (a.K) {
#define RPCA_CASE(KK)                                                                            \
    case KK:                                                                                     \
        hipLaunchKernelGGL((k_relax_stream<T, KK>), dim3(gs), dim3(RX_THREADS), 0, s, a);       \
        hipLaunchKernelGGL((k_relax_sum<KK>), dim3(gsum), dim3(256), 0, s, a);                   \
        hipLaunchKernelGGL((k_relax_gram<T, KK, true>), dim3(gpan), dim3(256), 0, s, a, (int)CNT_RELAX, a.gram);  \
        hipLaunchKernelGGL((k_relax_complement<T, KK>), dim3(gpan), dim3(256), 0, s, a);          \
        hipLaunchKernelGGL((k_relax_gram<T, KK, false>), dim3(gpan), dim3(256), 0, s, a, (int)CNT_RELAX, a.gram2); \
        hipLaunchKernelGGL((k_relax_tail<KK>), dim3(1), dim3(WAVE), 0, s, a);                    \
        hipLaunchKernelGGL((k_relax_update<T, KK>), dim3(gpan), dim3(256), 0, s, a);             \
        break;
        RPCA_CASE(1) RPCA_CASE(2) RPCA_CASE(3) RPCA_CASE(4) RPCA_CASE(5) RPCA_CASE(6)
        RPCA_CASE(7) RPCA_CASE(8) RPCA_CASE(9) RPCA_CASE(10)
#undef RPCA_CASE
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace

hipError_t launch_relax(const RelaxArgs& a, int dtype, hipStream_t s) {
    return dtype == 1 ? relax_dispatch<float>(a, s) : relax_dispatch<double>(a, s);
}

}  // namespace rpca
