// Tall-skinny (m x K, n x K) FP64 panel kernels between two streaming passes,
// and the small K x K / 2K x 2K FP64 linear algebra of Section 2.1.
//
// Row phases run one thread per row (four lanes per row in the gather) over
// the m rows of the U side and the n rows of the V side in one grid. Sums over
// rows (Grams, U_f^T Y1) are written as per-workgroup partials; the workgroup
// that arrives last (atomic counter + device-scope fences) keeps a single wave
// that sums them in a fixed order and runs the small dense algebra with
// wave-level synchronisation only, so results are deterministic and the
// serial tail has no block barriers.
//
// Notation (iteration k; K = r in the loop and K = p in the initialisation):
//   U_f, V_f   bases read by the streaming pass (dtype of D)
//   R_U, R_V   Cholesky factors of Gram(U_f), Gram(V_f); U* = U_f R_U^{-1},
//              V* = V_f R_V^{-1} are orthonormal to FP64 accuracy and span the
//              same spaces (a Cholesky QR whose R is applied implicitly), so
//              rounding the bases to FP32 never breaks the orthogonality the
//              2r x 2r reduction relies on
//   Y1 = Z V_f, Y2 = Z^T U_f                   (streaming pass, Z = D - S_k)
//   C*  = U*^T Z V*,  C2 = V*^T Z^T U*          (C2 = C*^T up to rounding)
//   W1  = (I - U* U*^T) Z V* = Q1 R1,  W2 = (I - V* V*^T) Z^T U* = Q2 R2
//   M   = [[C*, R2^T], [R1, 0]] = U_M Sigma_M V_M^T   (one-sided Jacobi)
//   U_{k+1} = [U* Q1] U_M[:, :K],  V_{k+1} = [V* Q2] V_M[:, :K]
// Q1, Q2 are never formed: U_{k+1} = U_f E1 + S_U E2 with small coefficient
// matrices, S_U = W1 (FP64 path) or Y1 (FP32 path, where Gram(W1) is formed
// as Gram(Y1*) - C*^T C*, exact to the FP32 level of the products).
#include "launch.hpp"
#include "wave.hpp"

namespace rpca {
namespace {

template <typename T> __device__ inline T* tptr(void* p) { return static_cast<T*>(p); }
template <typename T> __device__ inline const T* tptr(const void* p) { return static_cast<const T*>(p); }

// 16-byte vector of partial-sum values
template <typename A> struct Vec16;
template <> struct Vec16<float> { typedef float type __attribute__((ext_vector_type(4))); };
template <> struct Vec16<double> { typedef double type __attribute__((ext_vector_type(2))); };

// ---- row-phase helpers (whole workgroup) --------------------------------------

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

template <int K>
__device__ inline void block_load_small(const double* __restrict__ g, double* s) {
    for (int e = threadIdx.x; e < K * K; e += blockDim.x) s[e] = g[(e / K) * KMAX + (e % K)];
}

// Workgroup sum over NR row slots of a (x) b -> dst[t1 * K + t2] (global,
// K*K entries), for a workgroup of NT threads. Exactly one thread per slot
// passes writer = true (zero vectors for rows past the end). G adjacent lanes
// share an output entry: lane g of the group sums slots g, g + G, ..., then a
// fixed-order DPP reduction over the group (bitwise reproducible). sa, sb: LDS
// scratch of NR*K doubles each; every thread of the block must call it.
template <int K, int NR, int NT>
__device__ __forceinline__ void rows_outer_sum(const double (&a)[K], const double (&b)[K], bool writer, int slot, double* sa,
                               double* sb, double* __restrict__ dst) {
    constexpr int G0 = pow2_floor(NT / (K * K) > 0 ? NT / (K * K) : 1);
    constexpr int G = G0 > 16 ? 16 : G0;
    constexpr int STEP = NT / G;   // output entries handled at once
    if (writer) {
#pragma unroll
        for (int t = 0; t < K; ++t) {
            sa[slot * K + t] = a[t];
            sb[slot * K + t] = b[t];
        }
    }
    __syncthreads();
    const int sub = threadIdx.x % G;
    for (int e0 = threadIdx.x / G; e0 < (K * K + STEP - 1) / STEP * STEP; e0 += STEP) {
        const int e = e0 < K * K ? e0 : K * K - 1;   // whole groups stay in the loop for the DPP sum
        const int t1 = e / K, t2 = e % K;
        // four interleaved accumulators (shorter dependence chains), summed in a fixed order
        double c0 = 0.0, c1 = 0.0, c2 = 0.0, c3 = 0.0;
        int r = sub;
        for (; r + 3 * G < NR; r += 4 * G) {
            c0 = fma(sa[r * K + t1], sb[r * K + t2], c0);
            c1 = fma(sa[(r + G) * K + t1], sb[(r + G) * K + t2], c1);
            c2 = fma(sa[(r + 2 * G) * K + t1], sb[(r + 2 * G) * K + t2], c2);
            c3 = fma(sa[(r + 3 * G) * K + t1], sb[(r + 3 * G) * K + t2], c3);
        }
        for (; r < NR; r += G) c0 = fma(sa[r * K + t1], sb[r * K + t2], c0);
        double acc = (c0 + c1) + (c2 + c3);
        acc = group_sum<G>(acc);
        if (sub == 0 && e0 < K * K) dst[e] = acc;
    }
    __syncthreads();
}

// Two such sums with a shared right factor in one pass: dst1 = sum a1 (x) b,
// dst2 = sum a2 (x) b. sa1, sa2, sb: LDS scratch of NR*K doubles each.
template <int K, int NR, int NT>
__device__ __forceinline__ void rows_outer_sum2(const double (&a1)[K], const double (&a2)[K], const double (&b)[K],
                                                bool writer, int slot, double* sa1, double* sa2, double* sb,
                                                double* __restrict__ dst1, double* __restrict__ dst2) {
    constexpr int E = 2 * K * K;
    constexpr int G0 = pow2_floor(NT / E > 0 ? NT / E : 1);
    constexpr int G = G0 > 16 ? 16 : G0;
    constexpr int STEP = NT / G;
    if (writer) {
#pragma unroll
        for (int t = 0; t < K; ++t) {
            sa1[slot * K + t] = a1[t];
            sa2[slot * K + t] = a2[t];
            sb[slot * K + t] = b[t];
        }
    }
    __syncthreads();
    const int sub = threadIdx.x % G;
    for (int x0 = threadIdx.x / G; x0 < (E + STEP - 1) / STEP * STEP; x0 += STEP) {
        const int x = x0 < E ? x0 : E - 1;   // whole groups stay in the loop for the DPP sum
        const bool second = x >= K * K;
        const int e = second ? x - K * K : x;
        const double* sa = second ? sa2 : sa1;
        const int t1 = e / K, t2 = e % K;
        double c0 = 0.0, c1 = 0.0, c2 = 0.0, c3 = 0.0;
        int r = sub;
        for (; r + 3 * G < NR; r += 4 * G) {
            c0 = fma(sa[r * K + t1], sb[r * K + t2], c0);
            c1 = fma(sa[(r + G) * K + t1], sb[(r + G) * K + t2], c1);
            c2 = fma(sa[(r + 2 * G) * K + t1], sb[(r + 2 * G) * K + t2], c2);
            c3 = fma(sa[(r + 3 * G) * K + t1], sb[(r + 3 * G) * K + t2], c3);
        }
        for (; r < NR; r += G) c0 = fma(sa[r * K + t1], sb[r * K + t2], c0);
        double acc = (c0 + c1) + (c2 + c3);
        acc = group_sum<G>(acc);
        if (sub == 0 && x0 < E) (second ? dst2 : dst1)[e] = acc;
    }
    __syncthreads();
}

__device__ inline bool is_finite_pos(double x) { return x > 0.0 && x < 1e300; }
constexpr double MLP_O_CLIP = 5.0;   // the correction exp(o) stays within e^-5 .. e^5

// Output o of the threshold network (parameters th, FP32, layout of the
// training kernels) at features phi, evaluated in FP64 by one wave: lane j < 32
// owns hidden unit j. The result is valid in every lane. W2T: the second
// layer's weights are stored transposed (a copy in LDS, where lane j reading
// row j of the row-major matrix would put all 32 lanes on one bank).
template <bool W2T>
__device__ __forceinline__ double w_mlp(const float* __restrict__ th, const double (&phi)[MLP_IN]) {
    constexpr int OB1 = MLP_H * MLP_IN, OW2 = OB1 + MLP_H, OB2 = OW2 + MLP_H * MLP_H, OW3 = OB2 + MLP_H,
                  OB3 = OW3 + MLP_H;
    __shared__ double h1s[MLP_H];
    const int lane = lane_id();
    if (lane < MLP_H) {
        double v = th[OB1 + lane];
        for (int i = 0; i < MLP_IN; ++i) v = fma((double)th[lane * MLP_IN + i], phi[i], v);
        h1s[lane] = fmax(v, 0.0);
    }
    wave_sync();
    double c = 0.0;
    if (lane < MLP_H) {
        double v = th[OB2 + lane];
        for (int i = 0; i < MLP_H; ++i)
            v = fma((double)th[W2T ? OW2 + i * MLP_H + lane : OW2 + lane * MLP_H + i], h1s[i], v);
        c = (double)th[OW3 + lane] * fmax(v, 0.0);
    }
    for (int off = 32; off > 0; off >>= 1) c += __shfl_xor(c, off, WAVE);
    wave_sync();
    return c + (double)th[OB3];
}

// ---- the 2K x 2K step shared by the FP32 gather and the FP64 complement ------
//
// Single wave. Given C*, C2, the Grams G1 = W1^T W1 and G2 = W2^T W2 and
// R_U^{-1}, R_V^{-1}: R1, R2 by Cholesky, M = [[C*, R2^T], [R1, 0]], its SVD,
// then either the next threshold (Algorithm 1) or the convergence test of the
// initial subspace iteration, and the coefficients of the new factors
//   U_{k+1} = U_f E1 + S_U E2,   V_{k+1} = V_f F1 + S_V F2,
// with (S_U, S_V) = (Y1, Y2) when gram_form, (W1, W2) otherwise.
template <int K>
__device__ __forceinline__ void w_svd_tail(const PanelArgs& a, Ctrl* ctrl, const double* cs, const double* c2,
                           const double* g1, const double* g2, const double* ru, const double* rv,
                           bool gram_form, const float* th, bool th_lds) {
    constexpr int N = 2 * K;
    __shared__ double r1[K * K], r1i[K * K], r2[K * K], r2i[K * K];
    __shared__ double Ma[N * N], Mv[N * N], Um[N * N], Vm[N * N], sg[N];
    __shared__ double x1[K * K], x2[K * K], z1[K * K], z2[K * K], t1[K * K], t2[K * K];
    const int lane = lane_id();
    w_chol_inv2<K>(g1, r1, r1i, g2, r2, r2i);
    for (int e = lane; e < N * N; e += WAVE) {
        const int col = e / N, rw = e % N;
        double v = 0.0;
        if (rw < K && col < K) v = cs[rw * K + col];
        else if (rw < K) v = r2[(col - K) * K + rw];          // R2^T
        else if (col < K) v = r1[(rw - K) * K + col];         // R1
        Ma[e] = v;
    }
    wave_sync();
    // Pairs of columns with ||a||^2 <= sigma_dead^2 ||M||_F^2 / N <= (sigma_dead
    // sigma_1)^2 are not rotated against each other: both end below the
    // dropping level below, and such a rotation moves no other column.
    const double neg2 = ctrl->sigma_dead * ctrl->sigma_dead / N;
    const int sweeps = wave_jacobi_svd<N>(Ma, Mv, sg, Um, Vm, neg2, ctrl->single ? JACOBI_QUAD_F32 : JACOBI_QUAD);
    // Triplets whose singular value is at the rounding level of the products
    // (sigma_j <= sigma_dead * sigma_1) carry no information about the range
    // of P_T(Z): their vectors are noise and need not be orthogonal to U*, so
    // they are dropped (zero columns) instead of entering the next basis.
    const double cut = ctrl->sigma_dead * sg[0];
    for (int e = lane; e < N * N; e += WAVE) {
        if (sg[e / N] <= cut) { Um[e] = 0.0; Vm[e] = 0.0; }
    }
    wave_sync();
    // X1 = U_M[:K, :K], X2 = R1^{-1} U_M[K:, :K]; Z1, Z2 likewise from V_M
    for (int e = lane; e < K * K; e += WAVE) {
        const int i = e / K, j = e % K;   // coefficient row i, singular triplet j
        double xx = 0.0, zz = 0.0;
        for (int l = 0; l < K; ++l) {
            xx = fma(r1i[i * K + l], Um[j * N + K + l], xx);
            zz = fma(r2i[i * K + l], Vm[j * N + K + l], zz);
        }
        x1[e] = Um[j * N + i];
        z1[e] = Vm[j * N + i];
        x2[e] = xx;
        z2[e] = zz;
    }
    wave_sync();
    Small* sm = a.small;
    if (gram_form) {
        // E1 = R_U^{-1} (X1 - C* X2), E2 = R_V^{-1} X2, F1 = R_V^{-1} (Z1 - C2 Z2), F2 = R_U^{-1} Z2
        w_mm2<K, false>(cs, x2, t1, c2, z2, t2);
        for (int e = lane; e < K * K; e += WAVE) { t1[e] = x1[e] - t1[e]; t2[e] = z1[e] - t2[e]; }
        wave_sync();
        w_mm2<K, false>(ru, t1, x1, rv, t2, z1);
        w_mm2<K, false>(rv, x2, t1, ru, z2, t2);
        w_store<K>(x1, sm->E1);
        w_store<K>(t1, sm->E2);
        w_store<K>(z1, sm->F1);
        w_store<K>(t2, sm->F2);
    } else {
        // E1 = R_U^{-1} X1, E2 = X2, F1 = R_V^{-1} Z1, F2 = Z2
        w_mm2<K, false>(ru, x1, t1, rv, z1, t2);
        w_store<K>(t1, sm->E1);
        w_store<K>(x2, sm->E2);
        w_store<K>(t2, sm->F1);
        w_store<K>(z2, sm->F2);
    }
    if (lane < N) sm->sigma_M[lane] = sg[lane];
    if (lane < K) sm->sigma_new[lane] = sg[lane];
    // threshold network on the features of this iterate (whole wave)
    const bool use_mlp = ctrl->stage == STAGE_MAIN && ctrl->learned_on && th != nullptr;
    double mlp_o = 0.0;
    if (use_mlp) {
        const int r = ctrl->r;
        const double f = 1e-30;
        double phi[MLP_IN];
        phi[0] = (ctrl->k + 1) / MLP_K_FEAT;
        phi[1] = log(fmax(sg[r] / fmax(sg[0], f), MLP_SIGMA_RATIO_FLOOR));
        phi[2] = log(fmax(ctrl->err, f));
        phi[3] = log(fmax(sg[0], f) / fmax(sqrt(ctrl->normD2), f));
        mlp_o = th_lds ? w_mlp<true>(th, phi) : w_mlp<false>(th, phi);
    }
    if (lane == 0) {
        const int r = ctrl->r;
        if (ctrl->stage == STAGE_MAIN) {
            // zeta_{k+1} = beta (sigma_{r+1} + gamma^{k+1} sigma_1)  (Algorithm 1),
            // or the learned threshold while it is on (lane 0 has o in mlp_o)
            const int k = ctrl->k;
            const double s1 = sg[0], sr1 = sg[r];
            ctrl->sig1_pt = s1;
            ctrl->sigr1_pt = sr1;
            double z = ctrl->beta * (sr1 + pow(ctrl->gamma, (double)(k + 1)) * s1);
            if (use_mlp) {
                // learned correction of the paper's threshold: zeta * exp(clip(o))
                // (a NaN output must not reach fmin / fmax, which would clip it)
                const double zl = mlp_o == mlp_o ? z * exp(fmin(fmax(mlp_o, -MLP_O_CLIP), MLP_O_CLIP)) : NAN;
                if (is_finite_pos(zl)) z = zl;
                else ctrl->learned_on = 0;   // fallback: paper schedule from here on
            }
            ctrl->zeta = z;
            ctrl->k = k + 1;
        } else {
            // residual of the leading r directions of the previous block
            double acc = 0.0;
            for (int t = 0; t < r; ++t) acc += fmax(g1[t * K + t], 0.0) + fmax(g2[t * K + t], 0.0);
            const double res = sg[0] > 0.0 ? sqrt(acc) / sg[0] : 0.0;
            // res measures the block this pass started from; the block it
            // returns (the Ritz vectors of M) is better by about the contraction
            // factor of the iteration, estimated from the last two passes.
            // Converged: below the stage's tolerance; or that prediction for
            // the returned block, with a margin of 10, below it once the
            // iteration contracts steadily (third pass on, factor < 1/2), which
            // saves the pass that would only confirm it; or stalled (less than
            // a halving per pass) within 100x of it, where rounding of the
            // products limits the residual; or at the pass cap.
            const double rho = res / ctrl->res_prev;
            const bool steady = (ctrl->passes >= 3 || ctrl->res_carried) && rho < 0.5;
            const bool stall = ctrl->passes >= 3 && res > 0.5 * ctrl->res_prev;
            const bool capped = ctrl->passes >= ctrl->init_max_passes;
            const bool conv_a = res <= ctrl->tol_res_a || (steady && 10.0 * res * rho <= ctrl->tol_res_a) ||
                                (stall && res <= 100.0 * ctrl->tol_res_a) || capped;
            const bool conv_b = res <= ctrl->tol_res_b || (steady && 10.0 * res * rho <= ctrl->tol_res_b) ||
                                (stall && res <= 100.0 * ctrl->tol_res_b) || capped;
            const double res_last = res;
            ctrl->res_prev = res;
            if (ctrl->stage == STAGE_SIGMA_D && conv_a) {
                ctrl->sigma1_D = sg[0];
                const double z1 = ctrl->beta_init * sg[0];   // zeta_{-1} = beta_init sigma_1(D)
                ctrl->zeta = z1;
                // The stream passes compare |D_ij| > zeta in the precision of D.
                // When no entry exceeds zeta_{-1} there, S_{-1} is empty and
                // D - S_{-1} = D: the block already iterates on that matrix.
                const double zt = ctrl->single ? (double)(float)z1 : z1;
                const bool s_empty = ctrl->max_abs_D <= zt;
                if (s_empty && conv_b) {
                    ctrl->zeta = ctrl->beta * sg[0];      // zeta_0 = beta sigma_1(D - S_{-1})
                    ctrl->stage = STAGE_INIT_DONE;
                } else {
                    ctrl->stage = STAGE_INIT_Z;
                    ctrl->passes = 0;
                    ctrl->res_prev = s_empty ? res_last : 1e300;
                    ctrl->res_carried = s_empty ? 1 : 0;
                }
            } else if (ctrl->stage == STAGE_INIT_Z && conv_b) {
                ctrl->zeta = ctrl->beta * sg[0];          // zeta_0 = beta sigma_1(D - S_{-1})
                ctrl->stage = STAGE_INIT_DONE;
            }
        }
        ctrl->jacobi_sweeps += sweeps;
    }
    wave_sync();
}

// ---- kernel 1: gather partial products, C*, residual, stopping rule ----------
//
// NT threads, NT / 8 rows per workgroup (1024 and 128, or 512 and 64 for
// small problems: gather_threads_for; GATHER_SPLIT threads per row slot,
// the first of which holds the row): the per-tile partials of the
// workgroup's rows are summed with 16-byte loads of whole tile blocks, then
// the row products U_f^T Y1 (and Grams) are formed as workgroup partials.
// Instance blockIdx.y of a batched launch: every pointer of the arguments
// except the threshold network (shared) and the host status slot (unused in
// batches) moves by blockIdx.y * slab bytes.
__device__ inline PanelArgs at_instance(const PanelArgs& a0) {
    PanelArgs a = a0;
    if (a0.slab == 0) return a;
    const int64_t off = (int64_t)blockIdx.y * a0.slab;
    a.ctrl = shifted(a.ctrl, off);
    a.small = shifted(a.small, off);
    a.gpart = shifted(a.gpart, off);
    a.P1 = shifted(a.P1, off);
    a.P2 = shifted(a.P2, off);
    a.resid = shifted(a.resid, off);
    a.Y1 = shifted(a.Y1, off);
    a.Y2 = shifted(a.Y2, off);
    a.W1 = shifted(a.W1, off);
    a.W2 = shifted(a.W2, off);
    a.Ap = shifted(a.Ap, off);
    a.Bp = shifted(a.Bp, off);
    a.Unew = shifted(a.Unew, off);
    a.Vnew = shifted(a.Vnew, off);
    a.S2U = shifted(a.S2U, off);
    a.S2V = shifted(a.S2V, off);
    a.sigma_dst = shifted(a.sigma_dst, off);
    a.Uf = shifted(a.Uf, off);
    a.Vf = shifted(a.Vf, off);
    a.AL = shifted(a.AL, off);
    a.BL = shifted(a.BL, off);
    a.srcU = shifted(a.srcU, off);
    a.srcV = shifted(a.srcV, off);
    a.src_sigma = shifted(a.src_sigma, off);
    a.outU = shifted(a.outU, off);
    a.outV = shifted(a.outV, off);
    a.err_hist = shifted(a.err_hist, off);
    a.zeta_hist = shifted(a.zeta_hist, off);
    return a;
}

// The last workgroup sums the per-workgroup partials with all its threads.
// FP32 (gram_form): also the Grams of Y1 and Y2, and the whole 2K x 2K step in
// the tail. FP64: only C* and C2; the complement kernel forms W explicitly.
template <typename T, int K, int NT>
__global__ __launch_bounds__(NT) void k_gather(PanelArgs a_) {
    PanelArgs a = at_instance(a_);
    using Acc = typename AccOf<T>::type;
    constexpr int RPB = NT / GATHER_SPLIT;   // rows per workgroup
    constexpr bool GRAM = sizeof(T) == 4;
    Ctrl* ctrl = a.ctrl;
    // The gate is read here and tested once the tile sums are in LDS, so that
    // its latency overlaps the loads of the partials (which are harmless in a
    // body that does not run: they read the previous pass's partials).
    const bool runs = body_runs(ctrl, a.body);
    __shared__ int flag;
    const int gU = (a.m + RPB - 1) / RPB;
    const bool uside = (int)blockIdx.x < gU;
    const int slot = threadIdx.x / GATHER_SPLIT, chunk = threadIdx.x % GATHER_SPLIT;
    const int row0 = (uside ? blockIdx.x : blockIdx.x - gU) * RPB;
    const int row = row0 + slot;
    const int nrows = uside ? a.m : a.n;
    const int ntiles = uside ? a.n_ct : a.n_rt;
    const Acc* P = tptr<Acc>(uside ? a.P1 : a.P2);
    const bool holder = chunk == 0 && row < nrows;
    // the row of U_f (U side) or V_f (V side), and (rebuilding pass) of AL or
    // BL, loaded first and used last
    T fraw[K], lraw[K];
#pragma unroll
    for (int t = 0; t < K; ++t) fraw[t] = lraw[t] = T(0);
    if (holder) {
        const T* F = tptr<T>(uside ? a.Uf : a.Vf);
#pragma unroll
        for (int t = 0; t < K; ++t) fraw[t] = F[(size_t)row * K + t];
        if (a.lcorr) {
            const T* LF = tptr<T>(uside ? a.AL : a.BL);
#pragma unroll
            for (int t = 0; t < K; ++t) lraw[t] = LF[(size_t)row * K + t];
        }
    }
    // BL^T V_f (U side) or AL^T U_f (V side) for the rank-K part, one entry
    // per thread, put into LDS with the tile sums
    static_assert(K * K <= NT, "one entry of the cross product per thread");
    __shared__ double gk[K * K];
    double gkv = 0.0;
    if (a.lcorr && (int)threadIdx.x < K * K)
        gkv = (uside ? a.small->GBV : a.small->GAU)[(threadIdx.x / K) * KMAX + threadIdx.x % K];
    // Sum over the tiles of the streaming pass. Per tile, the rows of this
    // workgroup are one contiguous block of RPB * K values ([row][t]), read as
    // 16-byte vectors: NWG groups of NV threads each take every NWG-th tile
    // (up to LR loads in flight), and the groups' sums meet in LDS, summed in
    // group order (bitwise reproducible).
    constexpr int VW = 16 / (int)sizeof(Acc);
    constexpr int FB = RPB * K;
    constexpr int NV = FB / VW;
    constexpr int NWG = NT / NV;
    constexpr int LR = 8;
    static_assert(FB % VW == 0 && NWG >= 1, "tile block of the gather");
    typedef typename Vec16<Acc>::type VecT;
    // LDS: the groups' tile sums, later the row vectors of the products
    constexpr int NSH = NWG * FB > 3 * FB ? NWG * FB : 3 * FB;
    __shared__ double shbuf[NSH];
    double* gsum = shbuf;
    double* sa = shbuf;
    double* sb = shbuf + FB;
    {
        const int nval = (nrows - row0 < RPB ? nrows - row0 : RPB) * K;
        const size_t tstride = (size_t)nrows * K;
        const int grp = threadIdx.x / NV, vi = threadIdx.x % NV;
        double acc[VW];
#pragma unroll
        for (int j = 0; j < VW; ++j) acc[j] = 0.0;
        const Acc* base = P + (size_t)row0 * K + (size_t)vi * VW;
        if (grp < NWG && (vi + 1) * VW <= nval && tstride % VW == 0) {
            for (int c0 = grp; c0 < ntiles; c0 += LR * NWG) {
                VecT v[LR];
#pragma unroll
                for (int u = 0; u < LR; ++u) {
                    const int c = c0 + u * NWG;
                    v[u] = c < ntiles ? *reinterpret_cast<const VecT*>(base + (size_t)c * tstride) : VecT(0);
                }
#pragma unroll
                for (int u = 0; u < LR; ++u)
#pragma unroll
                    for (int j = 0; j < VW; ++j) acc[j] += static_cast<double>(v[u][j]);
            }
        } else if (grp < NWG) {
            // ragged end of the block, or a tile stride that is not a whole number of vectors
            for (int c = grp; c < ntiles; c += NWG)
#pragma unroll
                for (int j = 0; j < VW; ++j)
                    if (vi * VW + j < nval) acc[j] += static_cast<double>(base[(size_t)c * tstride + j]);
        }
        if (grp < NWG) {
#pragma unroll
            for (int j = 0; j < VW; ++j) gsum[grp * FB + vi * VW + j] = acc[j];
        }
    }
    if (a.lcorr && (int)threadIdx.x < K * K) gk[threadIdx.x] = gkv;
    if (!runs) {
        // A body queued past the end of its loop: the complement and update
        // kernels that follow read `active` and must do nothing either.
        // (The same decision in every workgroup: no barrier is left waiting.)
        if (blockIdx.x == 0 && threadIdx.x == 0) ctrl->active = 0;
        return;
    }
    __syncthreads();
    double y[K];
#pragma unroll
    for (int t = 0; t < K; ++t) y[t] = 0.0;
    if (chunk == 0 && row < nrows) {
        for (int g = 0; g < NWG; ++g)
#pragma unroll
            for (int t = 0; t < K; ++t) y[t] += gsum[g * FB + slot * K + t];
    }
    __syncthreads();   // gsum is reused as sa, sb below
    if (holder && a.lcorr) {
        // Y1 = E V_f + AL (BL^T V_f),  Y2 = E^T U_f + BL (AL^T U_f)
#pragma unroll
        for (int t = 0; t < K; ++t) {
            double c = 0.0;
#pragma unroll
            for (int u = 0; u < K; ++u) c = fma(static_cast<double>(lraw[u]), gk[u * K + t], c);
            y[t] += c;
        }
    }
    double f[K];
#pragma unroll
    for (int t = 0; t < K; ++t) f[t] = static_cast<double>(fraw[t]);   // zero unless holder
    if (holder) {
        double* Y = uside ? a.Y1 : a.Y2;
#pragma unroll
        for (int t = 0; t < K; ++t) Y[(size_t)row * K + t] = y[t];
    } else {
#pragma unroll
        for (int t = 0; t < K; ++t) y[t] = 0.0;
    }
    double* gp = a.gpart + (size_t)blockIdx.x * GPART_STRIDE;
    const bool writer = chunk == 0;   // y and f are zero unless this lane holds a valid row
    if (GRAM)   // U_f^T Y1 (V_f^T Y2) and Gram(Y1) (Gram(Y2))
        rows_outer_sum2<K, RPB, NT>(f, y, y, writer, slot, sa, shbuf + 2 * FB, sb, gp, gp + KMAX * KMAX);
    else
        rows_outer_sum<K, RPB, NT>(f, y, writer, slot, sa, sb, gp);   // U_f^T Y1 or V_f^T Y2
    if (!last_block_arrives(&ctrl->cnt[CNT_GATHER], &flag)) return;

    // ---- last workgroup: all threads sum the partials, then one wave ----
    __shared__ double sums[4 * K * K], ru[K * K], rv[K * K], cs[K * K], c2[K * K], tmp[K * K], tmp2[K * K];
    __shared__ double g1[K * K], g2[K * K];
    __shared__ double part[NT], rsum[2];
    double* craw = sums;              // U_f^T Y1
    double* craw2 = sums + K * K;     // V_f^T Y2
    double* gy1 = sums + 2 * K * K;   // Gram(Y1)
    double* gy2 = sums + 3 * K * K;   // Gram(Y2)
    const int gV = gridDim.x - gU;
    const bool sigma_stage = ctrl->stage == STAGE_SIGMA_D;
    // the residual tiles and R_U^{-1}, R_V^{-1} are loaded before the partials
    // are summed, so that the three loads overlap
    double rv_[RESID_LD], rw_[RESID_LD];
    block_resid_fetch<NT>(a.resid, a.n_tiles, sigma_stage, rv_, rw_);
    double ru_pre[w_per_lane<K>()], rv_pre[w_per_lane<K>()];
    if (threadIdx.x < WAVE) {
        w_fetch<K>(a.small->RUinv, ru_pre);
        w_fetch<K>(a.small->RVinv, rv_pre);
    }
    // The single-wave tail works on a copy of the control block in LDS (no
    // other workgroup or kernel touches it meanwhile), loaded with the other
    // loads of this phase and written back whole at the end.
    constexpr int CW = (int)(sizeof(Ctrl) / 4);
    static_assert(sizeof(Ctrl) % 4 == 0 && CW <= WAVE, "one word of the control block per lane");
    __shared__ Ctrl cl;
    uint32_t cword = 0;
    if (threadIdx.x < CW) cword = reinterpret_cast<const uint32_t*>(ctrl)[threadIdx.x];
    // The threshold network's parameters go to LDS for the tail (second
    // layer transposed, see w_mlp): loaded with this phase's other loads,
    // stored before the barrier of block_resid.
    __shared__ float th_s[GRAM ? MLP_PARAMS : 1];
    constexpr int TPT = GRAM ? (MLP_PARAMS + NT - 1) / NT : 1;
    float thv[TPT];
#pragma unroll
    for (int u = 0; u < TPT; ++u) {
        const int e = threadIdx.x + u * NT;
        thv[u] = (GRAM && a.mlp && e < MLP_PARAMS) ? a.mlp[e] : 0.f;
    }
    block_sum_partials<K * K, GRAM ? 4 : 2, NT>(a.gpart, gU, gV, sums, part);
#pragma unroll
    for (int u = 0; u < TPT; ++u) {
        const int e = threadIdx.x + u * NT;
        if (GRAM && a.mlp && e < MLP_PARAMS) {
            constexpr int OW2 = MLP_H * MLP_IN + MLP_H;
            const int w = e - OW2;
            th_s[(w >= 0 && w < MLP_H * MLP_H) ? OW2 + (w % MLP_H) * MLP_H + w / MLP_H : e] = thv[u];
        }
    }
    block_resid<NT>(a.resid, a.n_tiles, sigma_stage, rv_, rw_, part, rsum);
    if (threadIdx.x >= WAVE) return;
    const int lane = lane_id();
    if (lane < CW) reinterpret_cast<uint32_t*>(&cl)[lane] = cword;
    Ctrl* const cg = ctrl;   // the control block in device memory
    ctrl = &cl;
    w_put<K>(ru_pre, ru);
    w_put<K>(rv_pre, rv);
    // C* = R_U^{-T} (U_f^T Y1) R_V^{-1},  C2 = R_V^{-T} (V_f^T Y2) R_U^{-1}
    w_mm2<K, false>(craw, rv, tmp, craw2, ru, tmp2);
    w_mm2<K, true>(ru, tmp, cs, rv, tmp2, c2);
    w_store<K>(cs, a.small->Cstar);
    w_store<K>(c2, a.small->C2);
    const double rs = rsum[0], mx = rsum[1];
    int go_on = 0;
    if (lane == 0) {
        ctrl->resid2 = rs;
        if (sigma_stage) {
            ctrl->normD2 = rs;   // zeta = +inf: the residual is ||D||_F^2
            ctrl->max_abs_D = mx;
        }
        // A residual sum that is NaN or infinite comes from a non-finite entry
        // of D (or of the state a single step starts from); ||D||_F = 0 leaves
        // err_k = 0 / 0. Either ends the call: nothing queued after it runs.
        const bool bad = !(rs <= 1.7976931348623157e308) || (sigma_stage && !(rs > 0.0));
        if (bad) {
            ctrl->nonfinite = sigma_stage ? 1 : 2;
            ctrl->done = 1;
            ctrl->stopped_by_tol = 0;
            if (ctrl->stage != STAGE_MAIN) ctrl->stage = STAGE_FAILED;
        } else if (ctrl->stage == STAGE_MAIN) {
            const double err = sqrt(rs / ctrl->normD2);
            ctrl->err = err;
            const int k = ctrl->k;
            // learned schedule: fall back to the paper's once err stops decreasing
            if (ctrl->learned_on && k >= 1 && !(err < ctrl->err_prev)) ctrl->learned_on = 0;
            ctrl->err_prev = err;
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
        ctrl->cnt[CNT_GATHER] = 0;
        ctrl->post_update = 0;   // gpart now holds the gather's partials
        go_on = (GRAM && a.mode == GATHER_WITH_SVD && ctrl->active) ? 1 : 0;
    }
    go_on = __shfl(go_on, 0, WAVE);
    wave_sync();
    if (go_on) {
        // G1 = R_V^{-T} Gram(Y1) R_V^{-1} - C*^T C*,  G2 = R_U^{-T} Gram(Y2) R_U^{-1} - C2^T C2
        w_mm2<K, false>(gy1, rv, tmp, gy2, ru, tmp2);
        w_mm2<K, true>(rv, tmp, g1, ru, tmp2, g2);
        w_mm2<K, true>(cs, cs, craw, c2, c2, craw2);
        for (int e = lane; e < K * K; e += WAVE) { g1[e] -= craw[e]; g2[e] -= craw2[e]; }
        wave_sync();
        w_svd_tail<K>(a, ctrl, cs, c2, g1, g2, ru, rv, true, a.mlp ? th_s : nullptr, true);
    }
    wave_sync();
    if (lane < CW) reinterpret_cast<uint32_t*>(cg)[lane] = reinterpret_cast<const uint32_t*>(&cl)[lane];
}

// ---- kernel 2 (FP64): explicit complements W1, W2, their Grams, 2K x 2K step -

template <typename T, int K>
__global__ __launch_bounds__(PANEL_THREADS) void k_complement(PanelArgs a_) {
    PanelArgs a = at_instance(a_);
    Ctrl* ctrl = a.ctrl;
    if (!ctrl->active) return;
    __shared__ double sa[PANEL_THREADS * K], sb[PANEL_THREADS * K];
    __shared__ double ru[K * K], rv[K * K], cs[K * K], c2[K * K];
    __shared__ int flag;
    block_load_small<K>(a.small->RUinv, ru);
    block_load_small<K>(a.small->RVinv, rv);
    block_load_small<K>(a.small->Cstar, cs);
    block_load_small<K>(a.small->C2, c2);
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
        rowmul<K>(vs, c2, vc);     // V*_j C2
#pragma unroll
        for (int t = 0; t < K; ++t) { w[t] = ys[t] - vc[t]; a.W2[(size_t)row * K + t] = w[t]; }
    }
    rows_outer_sum<K, PANEL_THREADS, PANEL_THREADS>(w, w, true, threadIdx.x, sa, sb, a.gpart + (size_t)blockIdx.x * GPART_STRIDE);
    if (!last_block_arrives(&ctrl->cnt[CNT_COMPLEMENT], &flag)) return;
    __shared__ double gg[2 * K * K], part[PANEL_THREADS];
    double* g1 = gg;
    double* g2 = gg + K * K;
    block_sum_partials<K * K, 2, PANEL_THREADS>(a.gpart, a.gU, a.gV, gg, part);
    if (threadIdx.x >= WAVE) return;
    if (lane_id() == 0) ctrl->cnt[CNT_COMPLEMENT] = 0;
    w_svd_tail<K>(a, ctrl, cs, c2, g1, g2, ru, rv, false, a.mlp, false);
}

// ---- kernel 3: new factors (or entry from a given state), Trim, new bases ----
//
// Rows: U_{k+1} = U_f E1 + S_U E2 (or a given factor), the rebuild factors of
// L_{k+1}, Trim (Algorithm 2) and the basis for the next streaming pass,
// U_f = dtype(Trim(U_{k+1})); the Gram of the rounded values (FP64) gives R_U.
// Mode UPDATE_ENTER_EXACT keeps the FP64 trimmed factor and its Gram instead
// (FP64 orthonormal bases for rpca_trim).
template <typename T, int K>
__global__ __launch_bounds__(PANEL_THREADS) void k_update(PanelArgs a_) {
    PanelArgs a = at_instance(a_);
    Ctrl* ctrl = a.ctrl;
    const bool from_m = a.mode == UPDATE_FROM_M;
    if (a.body_id > 0 && blockIdx.x == 0 && threadIdx.x == 0) {
        // completion record of this body for the host (the control block is
        // final: the gather and complement kernels of the body have ended)
        volatile BodyRecord* rec = &a.host_status->body[a.body_id & (BODY_RING - 1)];
        rec->stage = ctrl->stage;
        rec->done = ctrl->done;
        rec->k = ctrl->k;
        rec->err = ctrl->err;
        __threadfence_system();
        rec->id = a.body_id;
        __threadfence_system();
    }
    // `active` is tested after the loads of this workgroup's rows are issued
    // (see below), so that the two latencies overlap.
    const bool skip = from_m && !ctrl->active;
    __shared__ double sa[PANEL_THREADS * K], sb[PANEL_THREADS * K], sc[PANEL_THREADS * K];
    __shared__ double e1[K * K], e2[K * K], sig[K];
    __shared__ int flag;
    const bool main_stage = !from_m || ctrl->stage == STAGE_MAIN;
    const bool uside = (int)blockIdx.x < a.gU;
    const int row = (uside ? blockIdx.x : blockIdx.x - a.gU) * PANEL_THREADS + threadIdx.x;
    const int nrows = uside ? a.m : a.n;
    T* F = tptr<T>(uside ? a.Uf : a.Vf);
    // All loads (the row's inputs, E1, E2, sigma) are issued before any of
    // them is used, so that their latencies overlap; raw values, converted
    // after the barrier.
    static_assert(K * K <= PANEL_THREADS, "one entry of E1, E2 per thread");
    const int tid = threadIdx.x;
    T fin[K];
    double in2[K];
#pragma unroll
    for (int t = 0; t < K; ++t) { fin[t] = T(0); in2[t] = 0.0; }
    if (row < nrows) {
        if (from_m) {
            const double* S2 = uside ? a.S2U : a.S2V;
#pragma unroll
            for (int t = 0; t < K; ++t) { fin[t] = F[(size_t)row * K + t]; in2[t] = S2[(size_t)row * K + t]; }
        } else {
            const double* src = uside ? a.srcU : a.srcV;
#pragma unroll
            for (int t = 0; t < K; ++t) in2[t] = src[(size_t)row * a.ld_src + t];
        }
    }
    double e1v = 0.0, e2v = 0.0, sgv = 1.0;
    if (from_m && tid < K * K) {
        const int at = (tid / K) * KMAX + tid % K;
        e1v = (uside ? a.small->E1 : a.small->F1)[at];
        e2v = (uside ? a.small->E2 : a.small->F2)[at];
    }
    if (tid < K) {
        if (from_m) sgv = a.small->sigma_new[tid];
        else if (a.src_sigma) sgv = a.src_sigma[tid];
    }
    if (tid < K * K) { e1[tid] = e1v; e2[tid] = e2v; }
    if (tid < K) sig[tid] = sgv;
    if (skip) return;   // the same in every workgroup
    __syncthreads();
    double gv[K], lf[K];   // the new basis row and the stored rebuild-factor row (zero past the end)
#pragma unroll
    for (int t = 0; t < K; ++t) gv[t] = lf[t] = 0.0;
    if (row < nrows) {
        double un[K];
        if (from_m) {
            double in1[K], p1[K], p2[K];
#pragma unroll
            for (int t = 0; t < K; ++t) in1[t] = static_cast<double>(fin[t]);
            rowmul<K>(in1, e1, p1);   // U_f E1
            rowmul<K>(in2, e2, p2);   // S_U E2
#pragma unroll
            for (int t = 0; t < K; ++t) un[t] = p1[t] + p2[t];
        } else {
#pragma unroll
            for (int t = 0; t < K; ++t) un[t] = in2[t];
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
            for (int t = 0; t < K; ++t) {
                const T v = static_cast<T>(uside ? un[t] * sig[t] : un[t]);
                LF[(size_t)row * K + t] = v;
                lf[t] = static_cast<double>(v);
            }
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
        if (a.mode == UPDATE_ENTER_EXACT) {
            double* Ap = uside ? a.Ap : a.Bp;
#pragma unroll
            for (int t = 0; t < K; ++t) { gv[t] = wgt * un[t]; Ap[(size_t)row * K + t] = gv[t]; }
        } else {
#pragma unroll
            for (int t = 0; t < K; ++t) {
                const T q = static_cast<T>(wgt * un[t]);
                F[(size_t)row * K + t] = q;
                gv[t] = static_cast<double>(q);
            }
        }
    }
    double* gp = a.gpart + (size_t)blockIdx.x * GPART_STRIDE;
    // Gram of the new basis; in the main stage (the next pass rebuilds L) also
    // AL^T U_f and BL^T V_f for the gather of the next pass
    if (main_stage)
        rows_outer_sum2<K, PANEL_THREADS, PANEL_THREADS>(gv, lf, gv, true, threadIdx.x, sa, sc, sb, gp, gp + KMAX * KMAX);
    else
        rows_outer_sum<K, PANEL_THREADS, PANEL_THREADS>(gv, gv, true, threadIdx.x, sa, sb, gp);
    if (from_m) {
        // Inside a loop the next kernel is a streaming pass; its workgroup 0
        // sums these partials (finish_basis) once its tile is done, off the
        // critical path: the results are first read by the gather after it.
        if (blockIdx.x == 0) {
            if (a.sigma_dst && threadIdx.x < K) a.sigma_dst[threadIdx.x] = sig[threadIdx.x];
            if (threadIdx.x == 0) ctrl->post_update = main_stage ? 2 : 1;
        }
        return;
    }
    if (!last_block_arrives(&ctrl->cnt[CNT_UPDATE], &flag)) return;
    __shared__ double fin_lds[FINISH_LDS<K, PANEL_THREADS>()];
    finish_basis<K, PANEL_THREADS, 32>(a.gpart, a.gU, a.gV, main_stage, a.mode == UPDATE_ENTER_EXACT, a.small,
                                       fin_lds);
    const int lane = lane_id();
    if (threadIdx.x < WAVE && a.sigma_dst && lane < K) a.sigma_dst[lane] = sig[lane];
    if (threadIdx.x == 0) {
        if (ctrl->stage == STAGE_INIT_DONE) ctrl->stage = STAGE_MAIN;
        ctrl->post_update = 0;   // nothing left for the next pass
        ctrl->cnt[CNT_UPDATE] = 0;
    }
}

// ---- cross products AL^T U_f, BL^T V_f of given factors and bases -----------
// For a rebuilding pass whose factors and bases were written elsewhere than by
// the update kernel (which forms the same products itself).
template <typename T, int K>
__global__ __launch_bounds__(PANEL_THREADS) void k_cross(PanelArgs a_) {
    PanelArgs a = at_instance(a_);
    Ctrl* ctrl = a.ctrl;
    __shared__ double sa[PANEL_THREADS * K], sb[PANEL_THREADS * K];
    __shared__ int flag;
    const bool uside = (int)blockIdx.x < a.gU;
    const int row = (uside ? blockIdx.x : blockIdx.x - a.gU) * PANEL_THREADS + threadIdx.x;
    const int nrows = uside ? a.m : a.n;
    double lf[K], f[K];
#pragma unroll
    for (int t = 0; t < K; ++t) lf[t] = f[t] = 0.0;
    if (row < nrows) {
        const T* LF = tptr<T>(uside ? a.AL : a.BL);
        const T* F = tptr<T>(uside ? a.Uf : a.Vf);
#pragma unroll
        for (int t = 0; t < K; ++t) {
            lf[t] = static_cast<double>(LF[(size_t)row * K + t]);
            f[t] = static_cast<double>(F[(size_t)row * K + t]);
        }
    }
    rows_outer_sum<K, PANEL_THREADS, PANEL_THREADS>(lf, f, true, threadIdx.x, sa, sb,
                                                    a.gpart + (size_t)blockIdx.x * GPART_STRIDE);
    if (!last_block_arrives(&ctrl->cnt[CNT_CROSS], &flag)) return;
    __shared__ double gg[2 * K * K], part[PANEL_THREADS];
    block_sum_partials<K * K, 2, PANEL_THREADS>(a.gpart, a.gU, a.gV, gg, part);
    if (threadIdx.x >= WAVE) return;
    w_store<K>(gg, a.small->GAU);
    w_store<K>(gg + K * K, a.small->GBV);
    if (lane_id() == 0) {
        ctrl->cnt[CNT_CROSS] = 0;
        ctrl->post_update = 0;   // gpart now holds these partials, not an update's
    }
}

// ---- FP64 orthonormal bases U~ = A R_A^{-1} of the trimmed factors ------------
// (rpca_trim's output; inside the loop the update kernel folds this step.)

template <typename T, int K>
__global__ __launch_bounds__(PANEL_THREADS) void k_basis(PanelArgs a_) {
    PanelArgs a = at_instance(a_);
    __shared__ double ri[K * K];
    const bool uside = (int)blockIdx.x < a.gU;
    block_load_small<K>(uside ? a.small->RAinv : a.small->RBinv, ri);
    __syncthreads();
    const int row = (uside ? blockIdx.x : blockIdx.x - a.gU) * PANEL_THREADS + threadIdx.x;
    const int nrows = uside ? a.m : a.n;
    if (row < nrows) {
        const double* Ap = uside ? a.Ap : a.Bp;
        double av[K], q[K];
#pragma unroll
        for (int t = 0; t < K; ++t) av[t] = Ap[(size_t)row * K + t];
        rowmul<K>(av, ri, q);
        double* out = uside ? a.outU : a.outV;
#pragma unroll
        for (int t = 0; t < K; ++t) out[(size_t)row * K + t] = q[t];
    }
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

template <typename T, int K>
__global__ __launch_bounds__(PANEL_THREADS) void k_start(PanelArgs a_) {
    PanelArgs a = at_instance(a_);
    Ctrl* ctrl = a.ctrl;
    __shared__ double sa[PANEL_THREADS * K], sb[PANEL_THREADS * K];
    __shared__ int flag;
    const bool uside = (int)blockIdx.x < a.gU;
    const int row = (uside ? blockIdx.x : blockIdx.x - a.gU) * PANEL_THREADS + threadIdx.x;
    const int nrows = uside ? a.m : a.n;
    double gv[K];
#pragma unroll
    for (int t = 0; t < K; ++t) gv[t] = 0.0;
    if (row < nrows) {
        T* F = tptr<T>(uside ? a.Uf : a.Vf);
        const uint64_t base = (uside ? 0ull : (uint64_t)a.m * K) + (uint64_t)row * K;
#pragma unroll
        for (int t = 0; t < K; ++t) {
            const T q = static_cast<T>(hash_uniform(a.seed, base + t));
            F[(size_t)row * K + t] = q;
            gv[t] = static_cast<double>(q);
        }
    }
    rows_outer_sum<K, PANEL_THREADS, PANEL_THREADS>(gv, gv, true, threadIdx.x, sa, sb, a.gpart + (size_t)blockIdx.x * GPART_STRIDE);
    if (!last_block_arrives(&ctrl->cnt[CNT_START], &flag)) return;
    __shared__ double gg[2 * K * K], rr[K * K], ri[K * K], rr2[K * K], ri2[K * K], part[PANEL_THREADS];
    double* g = gg;
    double* gb = gg + K * K;
    block_sum_partials<K * K, 2, PANEL_THREADS>(a.gpart, a.gU, a.gV, gg, part);
    if (threadIdx.x >= WAVE) return;
    w_chol_inv2<K>(g, rr, ri, gb, rr2, ri2);
    w_store<K>(ri, a.small->RUinv);
    w_store<K>(ri2, a.small->RVinv);
    if (lane_id() == 0) {
        ctrl->cnt[CNT_START] = 0;
        ctrl->post_update = 0;
    }
}

__global__ void k_setup(Ctrl* ctrl, Ctrl init, int64_t slab) {
    if (threadIdx.x == 0 && blockIdx.x == 0) *shifted(ctrl, (int64_t)blockIdx.y * slab) = init;
}

// The initialisation has converged and the entry update has run: switch the
// control block to the loop (stopping rule on, k = 0) on the device.
// (An instance of a batch whose initialisation failed keeps its state.)
__global__ void k_enter_loop(Ctrl* ctrl_, int64_t slab) {
    Ctrl* ctrl = shifted(ctrl_, (int64_t)blockIdx.y * slab);
    if (threadIdx.x == 0 && blockIdx.x == 0 && ctrl->stage != STAGE_FAILED) {
        ctrl->stage = STAGE_MAIN;
        ctrl->want_stop = 1;
        ctrl->k = 0;
        ctrl->active = 1;
        ctrl->done = 0;
        ctrl->err_prev = 1e300;
    }
}

// End of a solve: copies the control block and the leading hist_n entries of
// the err and zeta histories (at most k + 1 of them) into the call's status
// slot in mapped host memory, so that the host reads them after one stream
// synchronisation instead of three copies.
__global__ void k_publish(const Ctrl* ctrl, const double* err_hist, const double* zeta_hist, int hist_n,
                          HostStatus* dst) {
    constexpr int CW = (int)(sizeof(Ctrl) / 4);
    const uint32_t* src = reinterpret_cast<const uint32_t*>(ctrl);
    uint32_t* out = reinterpret_cast<uint32_t*>(&dst->fin);
    for (int i = threadIdx.x; i < CW; i += blockDim.x) out[i] = src[i];
    int n = ctrl->k + 1;
    if (n > hist_n) n = hist_n;
    if (n > PUBLISH_HIST) n = PUBLISH_HIST;
    for (int i = threadIdx.x; i < n; i += blockDim.x) {
        dst->hist[0][i] = err_hist[i];
        dst->hist[1][i] = zeta_hist[i];
    }
    __threadfence_system();
}

// Copies `bytes` (a multiple of 4) between each instance of a batch (instance
// blockIdx.x at slab0 + blockIdx.x * slab) and row blockIdx.x of a flat array
// (pitch bytes apart): to_slabs 1 writes the instances, 0 reads them.
__global__ void k_slab_copy(char* slab0, int64_t slab, char* flat, int64_t pitch, int64_t bytes, int to_slabs) {
    uint32_t* a = reinterpret_cast<uint32_t*>(slab0 + (int64_t)blockIdx.x * slab);
    uint32_t* b = reinterpret_cast<uint32_t*>(flat + (int64_t)blockIdx.x * pitch);
    for (int64_t w = threadIdx.x; w < bytes / 4; w += blockDim.x) {
        if (to_slabs) a[w] = b[w];
        else b[w] = a[w];
    }
}

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
#define RPCA_PANEL_LAUNCHER(NAME, GRID, BLOCK)                                                   \
    hipError_t NAME(const PanelArgs& a, int K, int dtype, hipStream_t s) {                       \
        const dim3 grid(GRID, a.batch > 1 ? (unsigned)a.batch : 1u), block(BLOCK);              \
        if (dtype == 1) { RPCA_K_SWITCH(RPCA_LAUNCH_F) } else { RPCA_K_SWITCH(RPCA_LAUNCH_D) }   \
        return hipGetLastError();                                                                \
    }

// The gather's workgroup size depends on the shape only (gather_threads_for),
// not on the number of instances of a batch.
#define RPCA_GATHER_F(KK) hipLaunchKernelGGL((k_gather<float, KK, NTG>), grid, block, 0, s, a)
#define RPCA_GATHER_D(KK) hipLaunchKernelGGL((k_gather<double, KK, NTG>), grid, block, 0, s, a)
template <int NTG>
hipError_t launch_gather_nt(const PanelArgs& a, int K, int dtype, hipStream_t s) {
    constexpr int rpb = NTG / GATHER_SPLIT;
    const dim3 grid((unsigned)((a.m + rpb - 1) / rpb + (a.n + rpb - 1) / rpb), a.batch > 1 ? (unsigned)a.batch : 1u),
        block(NTG);
    if (dtype == 1) { RPCA_K_SWITCH(RPCA_GATHER_F) } else { RPCA_K_SWITCH(RPCA_GATHER_D) }
    return hipGetLastError();
}
#undef RPCA_GATHER_F
#undef RPCA_GATHER_D

hipError_t launch_gather(const PanelArgs& a, int K, int dtype, hipStream_t s) {
    return gather_threads_for(a.m, a.n) == GATHER_THREADS_SMALL ? launch_gather_nt<GATHER_THREADS_SMALL>(a, K, dtype, s)
                                                                : launch_gather_nt<GATHER_THREADS>(a, K, dtype, s);
}
#define KFUN k_complement
RPCA_PANEL_LAUNCHER(launch_complement, (unsigned)(a.gU + a.gV), PANEL_THREADS)
#undef KFUN
#define KFUN k_update
RPCA_PANEL_LAUNCHER(launch_update, (unsigned)(a.gU + a.gV), PANEL_THREADS)
#undef KFUN
#define KFUN k_cross
RPCA_PANEL_LAUNCHER(launch_cross, (unsigned)(a.gU + a.gV), PANEL_THREADS)
#undef KFUN
#define KFUN k_basis
RPCA_PANEL_LAUNCHER(launch_basis, (unsigned)(a.gU + a.gV), PANEL_THREADS)
#undef KFUN
#define KFUN k_start
RPCA_PANEL_LAUNCHER(launch_start, (unsigned)(a.gU + a.gV), PANEL_THREADS)
#undef KFUN

hipError_t launch_setup(Ctrl* ctrl, const Ctrl& init, int batch, int64_t slab, hipStream_t s) {
    hipLaunchKernelGGL(k_setup, dim3(1, batch > 1 ? (unsigned)batch : 1u), dim3(64), 0, s, ctrl, init, slab);
    return hipGetLastError();
}

hipError_t launch_enter_loop(Ctrl* ctrl, int batch, int64_t slab, hipStream_t s) {
    hipLaunchKernelGGL(k_enter_loop, dim3(1, batch > 1 ? (unsigned)batch : 1u), dim3(64), 0, s, ctrl, slab);
    return hipGetLastError();
}

hipError_t launch_publish(const Ctrl* ctrl, const double* err_hist, const double* zeta_hist, int hist_n,
                          HostStatus* dst, hipStream_t s) {
    if (!dst || hist_n < 0) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_publish, dim3(1), dim3(128), 0, s, ctrl, err_hist, zeta_hist, hist_n, dst);
    return hipGetLastError();
}

hipError_t launch_slab_copy(void* slab0, int64_t slab, void* flat, int64_t pitch, int64_t bytes, int count,
                            int to_slabs, hipStream_t s) {
    if (count <= 0 || bytes <= 0 || (bytes & 3) || (pitch & 3) || (slab & 3)) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_slab_copy, dim3((unsigned)count), dim3(256), 0, s, static_cast<char*>(slab0), slab,
                       static_cast<char*>(flat), pitch, bytes, to_slabs);
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
