// Shared definitions of librpca: workspace control block, small FP64 matrix
// area, launch constants and device helpers used by several kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <type_traits>

namespace rpca {

constexpr int KMAX = 16;          // largest rank / init block handled by the kernels
constexpr int WAVE = 64;          // CDNA wavefront width
constexpr int STREAM_THREADS = 256;
constexpr int STREAM_WAVES = STREAM_THREADS / WAVE;
constexpr int STREAM_CPL = 4;     // consecutive columns owned by one lane
constexpr int STREAM_TN = WAVE * STREAM_CPL;   // columns per stream tile
constexpr int PANEL_THREADS = 256;
constexpr int GATHER_SPLIT = 8;   // adjacent lanes sharing one row in the gather kernel (<= 16)
constexpr int GATHER_THREADS = 1024;        // gather workgroup: 128 rows
constexpr int GATHER_THREADS_SMALL = 512;   // gather workgroup for small problems: 64 rows
constexpr int GATHER_SMALL_MAX_ROWS = 8192; // m + n up to which the small workgroup is used
// Threads per workgroup of the gather kernel for an m x n problem. Halving the
// rows per workgroup below m + n = 8192 spreads the small problems' partial
// sums over twice as many CUs (2-3 % faster solves at m = n = 2000-3000, 7 %
// for a batch of 2000 x 2000 instances); above, the last workgroup's sum over
// the doubled number of partials costs more than that gains.
__host__ __device__ constexpr int gather_threads_for(int64_t m, int64_t n) {
    return m + n <= GATHER_SMALL_MAX_ROWS ? GATHER_THREADS_SMALL : GATHER_THREADS;
}
constexpr int GPART_STRIDE = 2 * KMAX * KMAX;   // doubles per workgroup partial slot
// relaxed iteration (threshold training)
constexpr int RX_KMAX = 10;        // largest rank of the relaxed iteration (3r <= 30 for the wave SVD)
constexpr int RX_TRUE_MAX = 16;    // largest rank of the loss's target factors
constexpr int RX_THREADS = 256;    // columns per tile of its pass over D (one per thread)
constexpr int RX_MAX_RT = 16;      // row tiles of that pass
constexpr int RX_WMAX = 3 * RX_KMAX + RX_TRUE_MAX;   // widest Gram, [F Y dY P]
// threshold network: phi (4) -> 32 -> 32 -> 1
constexpr int MLP_IN = 4, MLP_H = 32;
constexpr int MLP_PARAMS = MLP_H * MLP_IN + MLP_H + MLP_H * MLP_H + MLP_H + MLP_H + 1;   // 1249
constexpr double MLP_K_FEAT = 15.0;   // iteration count that normalises the first feature
// sigma_{r+1} / sigma_1 enters the features clamped from below: the FP32 path
// resolves sigma_{r+1} only to about 1e-5 sigma_1, so smaller ratios are noise
constexpr double MLP_SIGMA_RATIO_FLOOR = 1e-4;

// Stages of the device-side state machine (Ctrl::stage).
enum Stage : int {
    STAGE_SIGMA_D = 0,   // init: subspace iteration on D for sigma_1(D)
    STAGE_INIT_Z = 1,    // init: subspace iteration on D - T_{zeta_-1}(D)
    STAGE_INIT_DONE = 2, // init converged; host switches to rank-r kernels
    STAGE_MAIN = 3,      // AccAltProj loop
    STAGE_FAILED = 4,    // init stopped: ||D||_F = 0 or a non-finite entry in D
};

// Which loop a kernel launch belongs to (gating of speculatively queued bodies).
enum Body : int {
    BODY_INIT = 0,   // runs only while the initial subspace iteration is in progress
    BODY_MAIN = 1,   // runs only while the AccAltProj loop has not stopped
    BODY_ANY = 2,    // always runs (single steps, tests)
};

// Counter slots for the last-workgroup-finishes pattern.
enum CounterSlot : int {
    CNT_GATHER = 0, CNT_COMPLEMENT = 1, CNT_UPDATE = 2, CNT_BASIS = 3, CNT_START = 4, CNT_RELAX = 5, CNT_CROSS = 6,
    CNT_COUNT = 8,
};

// Completion record of one queued body, written into mapped host memory by
// the body's last kernel (ring slot id & (BODY_RING - 1)); id is written last.
struct BodyRecord {
    int32_t id;          // body id given by the host (> 0)
    int32_t stage;
    int32_t done;        // loop finished
    int32_t k;
    double err;          // err of the state the body started from (loop bodies)
};
constexpr int BODY_RING = 8;

// Control block at the start of the workspace (device memory).
struct Ctrl {
    uint32_t cnt[CNT_COUNT];
    int32_t done;        // main loop finished (err < tol or k == max_iter)
    int32_t stage;
    int32_t k;           // index of the current state (L_k, S_k)
    int32_t passes;      // passes over D in the current init stage
    int32_t total_passes;
    int32_t max_iter;
    int32_t keep;        // singular triplets kept from M (p in init, r in main)
    int32_t r;
    int32_t p;
    int32_t init_max_passes;
    int32_t trim;        // 1: apply Algorithm 2 in the update kernel
    int32_t want_stop;   // 1: gather kernel applies the stopping rule
    int32_t stopped_by_tol;
    int32_t active;      // 1 while the current loop body is live (set by the gather kernel)
    int32_t jacobi_sweeps;   // sweeps of the last 2K x 2K SVD (diagnostic)
    int32_t post_update; // 1 (Gram only) or 2 (Gram and cross products): the update kernel left
                         // the sums of its partials to workgroup 0 of the next streaming pass
    double zeta;         // threshold used by the next stream pass
    double err;          // err of the current state
    double normD2;       // ||D||_F^2
    double beta, beta_init, gamma, mu, tol;
    double res_prev;     // init convergence tracking
    double sigma1_D;
    double sig1_pt, sigr1_pt;   // sigma_1 and sigma_{r+1} of the last P_T(D - S_k)
    double tol_res_a, tol_res_b;
    double resid2;       // last residual sum (sum over |x| <= zeta of x^2)
    double sigma_dead;   // relative size below which a singular triplet of M is dropped
    double max_abs_D;    // max |D_ij| (from the init passes, where L = 0)
    double err_prev;     // err_{k-1} (fallback test of the learned schedule)
    int32_t learned_on;  // 1 while zeta_{k+1} comes from the threshold network
    int32_t res_carried; // 1: the init stage continues the previous stage's iteration (res_prev is its)
    int32_t single;      // 1: D and the streamed factors are FP32
    int32_t nonfinite;   // 1: ||D||_F^2 was zero or not finite (bad input);
                         // 2: a later residual sum was not finite (bad state or breakdown)
};

// Leading entries of the err and zeta histories that a solve's last kernel
// copies into its status slot; a longer history is read with two copies.
constexpr int PUBLISH_HIST = 128;
// One per call in flight on a device (a pool in mapped, coherent host memory).
struct HostStatus {
    BodyRecord body[BODY_RING];
    Ctrl fin;                        // control block at the end of a solve
    double hist[2][PUBLISH_HIST];    // err_0.., zeta_0.. at the end of a solve
};

// Small FP64 matrices shared between kernels (all K x K, row-major, ld = KMAX).
struct Small {
    double RUinv[KMAX * KMAX];   // R_U^{-1}: Gram(U_f) = R_U^T R_U
    double RVinv[KMAX * KMAX];
    double Cstar[KMAX * KMAX];   // C* = R_U^{-T} U_f^T Y1 R_V^{-1}
    double C2[KMAX * KMAX];      // C2 = R_V^{-T} V_f^T Y2 R_U^{-1}  (= C*^T up to rounding)
    double E1[KMAX * KMAX];      // U_new = U_f E1 + S_U E2  (S_U = Y1 or W1)
    double E2[KMAX * KMAX];
    double F1[KMAX * KMAX];      // V_new = V_f F1 + S_V F2  (S_V = Y2 or W2)
    double F2[KMAX * KMAX];
    double RAinv[KMAX * KMAX];   // Gram(A) = R_A^T R_A (Trim output)
    double RBinv[KMAX * KMAX];
    double sigma_new[KMAX];
    double sigma_M[2 * KMAX];
    // Cross products of the rebuild factors with the bases of a streaming
    // pass: GAU = AL^T U_f, GBV = BL^T V_f (products of the stored values).
    // With Z = D - S = L + E, E = D - L - S, the pass forms E V_f and E^T U_f
    // and the gather adds L V_f = AL GBV and L^T U_f = BL GAU.
    double GAU[KMAX * KMAX];
    double GBV[KMAX * KMAX];
};

__host__ __device__ constexpr size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

// ---------------------------------------------------------------- device --

template <typename T> struct AccOf;
template <> struct AccOf<float> { using type = float; };
template <> struct AccOf<double> { using type = double; };

// Sum of one double over the threads of a workgroup (result valid in all
// threads; fixed order). red: shared scratch of blockDim.x / 64 doubles.
__device__ inline double block_sum(double v, double* red) {
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, WAVE);
    const int w = threadIdx.x / WAVE;
    const int nw = blockDim.x / WAVE;
    __syncthreads();
    if ((threadIdx.x & (WAVE - 1)) == 0) red[w] = v;
    __syncthreads();
    double s = 0.0;
    for (int i = 0; i < nw; ++i) s += red[i];
    __syncthreads();
    return s;
}
__device__ inline double block_sum_256(double v, double* red) { return block_sum(v, red); }

// Whether a streaming pass / gather launch of the given body executes.
__device__ inline bool body_runs(const Ctrl* c, int body) {
    if (body == BODY_INIT) return c->stage == STAGE_SIGMA_D || c->stage == STAGE_INIT_Z;
    if (body == BODY_MAIN) return c->done == 0;
    return true;
}

// Signals completion of this workgroup's partial results; returns true in all
// threads of the single workgroup that finished last. Partials written by any
// thread of any workgroup before the call are visible to that workgroup
// afterwards. The counter is reset by the caller.
// Thread 0 alone issues the agent-scope fences, after a workgroup barrier
// (which completes every wave's stores at workgroup scope; the release fence
// is cumulative over them) and before the barrier that hands the result to the
// other waves. A fence in every wave multiplies the L2 write-backs.
// Tile handled by workgroup b of a G-workgroup launch. Workgroups are handed to
// the 8 XCDs of the device in turn (b, b + 8, ... on XCD b % 8); numbering the
// tiles so that each XCD takes one contiguous run puts neighbouring tiles
// (the column tiles of a row band, which share the cache lines at their
// edges) on one XCD and its L2. A bijection of 0..G-1.
__device__ inline int xcd_tile(int b, int G) {
    constexpr int NX = 8;
    const int q = G / NX, rm = G % NX;
    const int x = b % NX, pos = b / NX;
    return (x < rm ? x * (q + 1) : rm * (q + 1) + (x - rm) * q) + pos;
}

// Loads of D, which every pass reads exactly once. NT: marked non-temporal, so
// that streaming the m x n data does not evict from the L2 what the kernels
// around the pass reuse (bases, partial sums, code). Measured at
// m = n = 10^4, r = 5: FP32 loop pass 97.2 -> 95.6 us, initialisation pass
// 98.2 -> 94.8 us, loop body 147.9 -> 144.2 us; at m = n = 2 10^4, r = 10,
// where the pass is bound by its vector ALU work, the loop pass went from
// 641 to 675 us, and FP64 passes (8-byte D) were slower with them at every
// size measured (m = n = 5000: solve 2.09 -> 2.43 ms). Passes over FP32 D use
// them for blocks of up to D_LOADS_NT_KMAX columns.
constexpr int D_LOADS_NT_KMAX = 6;
typedef float nt_float4 __attribute__((ext_vector_type(4)));
typedef double nt_double2 __attribute__((ext_vector_type(2)));
template <bool NT> __device__ inline float4 load_d(const float4* p) {
    if constexpr (!NT) return *p;
    const nt_float4 v = __builtin_nontemporal_load(reinterpret_cast<const nt_float4*>(p));
    return make_float4(v.x, v.y, v.z, v.w);
}
template <bool NT> __device__ inline double2 load_d(const double2* p) {
    if constexpr (!NT) return *p;
    const nt_double2 v = __builtin_nontemporal_load(reinterpret_cast<const nt_double2*>(p));
    return make_double2(v.x, v.y);
}
template <bool NT> __device__ inline float load_d(const float* p) {
    if constexpr (!NT) return *p;
    return __builtin_nontemporal_load(p);
}
template <bool NT> __device__ inline double load_d(const double* p) {
    if constexpr (!NT) return *p;
    return __builtin_nontemporal_load(p);
}

// p moved by off bytes (the data of another instance of a batched launch);
// a null pointer stays null.
template <typename X> __device__ inline X* shifted(X* p, int64_t off) {
    return p ? reinterpret_cast<X*>(reinterpret_cast<uintptr_t>(p) + (uintptr_t)off) : p;
}
// The same for a pointer that is never null, as plain address arithmetic
// (keeps a kernel argument in scalar registers).
template <typename X> __device__ inline X* moved(X* p, int64_t off) {
    using C = typename std::conditional<std::is_const<X>::value, const char, char>::type;
    return reinterpret_cast<X*>(reinterpret_cast<C*>(p) + off);
}

// Last-workgroup election. The workgroup barrier orders the waves but does not
// wait for their global stores to complete (only for their LDS operations),
// and the increment's release (agent scope: write-back of this XCD's L2, then
// the atomic) covers what has reached the L2 by then. So every wave first
// waits until its own stores have completed, i.e. reached the L2; otherwise
// a partial still in flight from another wave could miss the write-back, and
// the last workgroup, on another XCD with its own L2, would read a stale
// value. (A release fence in every wave would also do, at 16 L2 write-backs
// per workgroup: 17 us more per loop body at m = n = 10^4.) Only the last
// workgroup acquires, so the others skip the L2 invalidation a full fence
// costs.
__device__ inline bool last_block_arrives(uint32_t* counter, int* flag_smem) {
    __asm__ volatile("s_waitcnt vmcnt(0)" ::: "memory");
    __syncthreads();
    if (threadIdx.x == 0) {
        const uint32_t prev = __hip_atomic_fetch_add(counter, 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
        const int last = (prev == gridDim.x - 1) ? 1 : 0;
        if (last) __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
        *flag_smem = last;
    }
    __syncthreads();
    return *flag_smem != 0;
}

}  // namespace rpca
