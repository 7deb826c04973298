// Host-side launchers of the librpca kernels (defined next to the kernels).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "common.hpp"

namespace rpca {

// Arguments of the streaming pass over D (see stream.hip).
struct StreamArgs {
    const void* D;        // m x n, row stride ldd (T)
    int64_t ldd;
    int32_t m, n;
    const void* AL;       // m x K (T): L = AL BL^T ; unused without rebuild
    const void* BL;       // n x K (T)
    const void* Uf;       // m x K (T): basis for Y2 = Z^T Uf
    const void* Vf;       // n x K (T): basis for Y1 = Z Vf
    Ctrl* ctrl;           // zeta, done (read); post_update, cnt (completing an update)
    void* P1;             // [n_ct][m][K] partials of Y1 (acc type)
    void* P2;             // [n_rt][n][K] partials of Y2
    double* resid;        // [n_ct * n_rt] partial residual sums
    int32_t TM;           // rows per tile
    int32_t n_ct, n_rt;
    int32_t vec_ok;       // 1 if D rows are 16-byte aligned (vector loads allowed)
    int32_t body;         // Body: gating of the launch
    int32_t batch;        // instances in the launch (grid y); every pointer above is
    int64_t slab;         // instance 0's, instance i's lies i * slab bytes further
    // The update kernel's closing sums, left to this pass (ctrl->post_update):
    double* post_gpart;   // its per-workgroup partials (gU + gV slots)
    Small* post_small;    // destination of R_U^{-1}, R_V^{-1}, A_L^T U_f, B_L^T V_f
    int32_t post_gU, post_gV;
};

// Scalar geometry of the streaming pass (kernel argument; pointers are passed
// separately so the compiler can treat them as non-aliasing).
struct StreamGeom {
    int64_t ldd;
    int32_t m, n, TM, n_ct, n_rt, vec_ok, body;
    int64_t slab;         // bytes between the instances of a batched launch (0: one instance)
    double* post_gpart;   // see StreamArgs (null: the pass never completes an update)
    Small* post_small;
    int32_t post_gU, post_gV;
};

struct MaterializeArgs {
    const void* D;
    int64_t ldd;
    int32_t m, n;
    const void* AL;
    const void* BL;
    const Ctrl* ctrl;
    void* L_out; int64_t ldl;
    void* S_out; int64_t lds;
};

// Panel-kernel arguments (one struct for all of them; unused fields ignored).
struct PanelArgs {
    int32_t m, n;
    int32_t gU, gV;           // workgroups on the U side (m rows) and V side (n rows)
    Ctrl* ctrl;
    Small* small;
    double* gpart;            // per-workgroup partial K x K blocks [gU + gV][KMAX*KMAX]
    // stream partials
    const void* P1; const void* P2; int32_t n_ct, n_rt;
    const double* resid; int32_t n_tiles;
    // FP64 panels
    double* Y1; double* Y2;   // m x K, n x K
    double* W1; double* W2;
    double* Ap; double* Bp;   // trimmed factors / blocks to orthonormalise
    double* Unew; double* Vnew;  // destinations of the updated factors (stride K)
    const double* S2U; const double* S2V;  // second panels of the update (Y or W)
    double* sigma_dst;        // destination of sigma_new (nullable)
    // T-typed panels
    void* Uf; void* Vf;       // bases used by the stream pass
    void* AL; void* BL;       // rebuild factors
    // enter mode sources
    const double* srcU; const double* srcV; int64_t ld_src; const double* src_sigma;
    // optional FP64 outputs of the basis kernel
    double* outU; double* outV;
    // histories and host status
    double* err_hist; double* zeta_hist; int32_t hist_cap;
    HostStatus* host_status;  // the call's status slot (device view), or null
    int32_t body_id;          // update kernel: > 0 writes the body's completion record
    uint64_t seed;
    const float* mlp;         // threshold network parameters (learned schedule) or null
    int32_t mode;             // kernel-specific
    int32_t body;             // Body of the gather kernel
    int32_t gated;            // basis kernel: skip when the body is not active
    int32_t batch;            // instances in the launch (grid y), 0 or 1: one
    int64_t slab;             // bytes between instances: every pointer but mlp and host_status
                              // is instance 0's and is moved by blockIdx.y * slab
    int32_t lcorr;            // gather: the pass rebuilt L; add AL GBV to Y1 and BL GAU to Y2
};

// Results of one relaxed iteration (device, written by its tail kernel).
struct RelaxResult {
    double loss, dloss_dzeta;   // ||L_{k+1} - P Q^T||^2 / ||P Q^T||^2 and its zeta-derivative
    double err;                 // ||x - s(x)||_F / ||D||_F at L_k (relaxed err_k)
    double sigma1, sigma_r1;    // sigma_1 and sigma_{r+1} of P_T(Z)
    int32_t sweeps, pad;
};

// Arguments of the relaxed iteration's kernels (see relax.hip).
struct RelaxArgs {
    const void* D; int64_t ldd;
    int32_t m, n, K, rt_true;
    const void* AL; const void* BL; const void* Uf; const void* Vf;
    double zeta, tau, normD2;
    int32_t TM, n_ct, n_rt, n_tiles, gU, gV;
    double* R1; double* R2; double* Rres;   // per-tile partials [n_ct][m][2K], [n_rt][n][2K]
    double* RY1; double* RY2;               // [Y1 dY1] (m x 2K), [Y2 dY2] (n x 2K)
    double* gpartR;                         // Gram partials
    double* gram;  double* gram2;           // [F Y dY P] and [W dW P] Grams, U side then V side
    const double* P; const double* Q;       // target factors, m x rt_true and n x rt_true
    const double* RUinv; const double* RVinv;
    double* coef;                           // 6 K x K coefficient blocks of the new factors
    double* sigma_out; double* Uout; double* Vout;
    RelaxResult* result;
    Ctrl* ctrl;
};

enum UpdateMode : int { UPDATE_FROM_M = 0, UPDATE_ENTER = 1, UPDATE_ENTER_EXACT = 2 };
enum GatherMode : int { GATHER_ONLY = 0, GATHER_WITH_SVD = 1 };

// dtype: 0 = double, 1 = float
// Workgroups of the streaming pass resident per CU (from the HIP occupancy API).
int stream_occupancy(int K, int dtype, bool rebuild);
int stream_mx_occupancy(int K, bool rebuild);
hipError_t launch_stream_mx(const StreamArgs& a, int K, bool rebuild, hipStream_t s);
hipError_t launch_stream(const StreamArgs& a, int K, int dtype, bool rebuild, hipStream_t s);
hipError_t launch_materialize(const MaterializeArgs& a, int K, int dtype, hipStream_t s);
hipError_t launch_read_probe(const void* data, int64_t bytes, float* sink, int blocks, hipStream_t s);
hipError_t launch_gather(const PanelArgs& a, int K, int dtype, hipStream_t s);
hipError_t launch_complement(const PanelArgs& a, int K, int dtype, hipStream_t s);
hipError_t launch_update(const PanelArgs& a, int K, int dtype, hipStream_t s);
hipError_t launch_cross(const PanelArgs& a, int K, int dtype, hipStream_t s);
hipError_t launch_basis(const PanelArgs& a, int K, int dtype, hipStream_t s);
hipError_t launch_start(const PanelArgs& a, int K, int dtype, hipStream_t s);
hipError_t launch_setup(Ctrl* ctrl, const Ctrl& init, int batch, int64_t slab, hipStream_t s);
hipError_t launch_enter_loop(Ctrl* ctrl, int batch, int64_t slab, hipStream_t s);
hipError_t launch_publish(const Ctrl* ctrl, const double* err_hist, const double* zeta_hist, int hist_n,
                          HostStatus* dst, hipStream_t s);
hipError_t launch_slab_copy(void* slab0, int64_t slab, void* flat, int64_t pitch, int64_t bytes, int count,
                            int to_slabs, hipStream_t s);
hipError_t launch_relax(const RelaxArgs& a, int dtype, hipStream_t s);

// Reverse mode of unrolled relaxed iterations (adjoint.hip).
struct AdjointProblem {
    const void* D;
    int64_t ldd, m, n;
    int32_t dtype, K, Kt, rt;                 // rank, bodies, rank of the target factors
    const double* P;                          // target factors, m x rt and n x rt
    const double* Q;
    const double* const* U;                   // host arrays of Kt + 1 device checkpoints
    const double* const* sigma;
    const double* const* V;
    const double* zeta;                       // host arrays of Kt
    const double* tau;
    const double* weight;
    double cU, cV;                            // trim levels (0: no trim)
    int32_t TM, n_ct, n_rt;                   // tiling of the passes over D
    double* zeta_bar_dev;                     // device outputs
    double* U_bar;
    double* sigma_bar;
    double* V_bar;
};
struct AdjointBufs {
    struct Slot {
        double *Am, *wU, *rhoU, *BU, *Bm, *wV, *rhoV, *BV;
        double *RAinv, *RBinv, *C, *R1, *R2, *R1inv, *R2inv, *UM, *SM, *VM;
    } slot[2];
    double *Y1, *W1, *GammaV, *YG, *SR, *GU, *Abar, *Utrim, *F1;
    double *Y2, *W2, *GammaU, *XG, *SC, *GV, *Bbar, *Vtrim, *F2;
    double *Rp, *Cp, *scal, *scal_out, *gpart, *small;
    double* zbar;                             // dloss/dzeta_k, RPCA_MAX_UNROLL values
    uint32_t* cnt;
    char* end;
};
size_t adjoint_ws_bytes(int64_t m, int64_t n, int K, int n_ct, int n_rt);
hipError_t adjoint_carve(void* base, int64_t m, int64_t n, int K, int n_ct, int n_rt, AdjointBufs* b);
hipError_t adjoint_run(const AdjointProblem& P, const AdjointBufs& B, hipStream_t s);
hipError_t launch_mlp_forward(const float* th, const float* phi, float* o, int B, hipStream_t s);
hipError_t launch_mlp_backward(const float* th, const float* phi, const float* g, int B, float* grad, hipStream_t s);
hipError_t launch_mlp_adam(float* th, float* m, float* v, const float* g, int t, float lr, float b1, float b2,
                           float eps, hipStream_t s);
hipError_t launch_convert(const double* src, void* dst, int64_t count, const double* scale, int K,
                          int dtype, hipStream_t s);

}  // namespace rpca
