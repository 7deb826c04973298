// The streaming pass with both tangent products on the matrix cores (the
// mixed-precision form). Per element of D, in FP32 on the vector ALUs, as in
// the FP32 pass: the rank-K rebuild of L, the threshold T_zeta, the residual
// part E = D - L - S (Section 2.1 and Algorithm 1) and its square. E is
// rounded to BF16 into LDS, and both products of the residual part run on the
// matrix cores with FP32 accumulation: E V_f (the row sums, which on the vector
// ALUs cost a cross-lane reduction per row) and E^T U_f (the column sums), with
// V_f and U_f rounded to BF16 too. As in the FP32 pass, the gather adds the
// rank-K parts L V_f and L^T U_f exactly, so only the products of E carry the
// BF16 rounding (~2^-9 relative per term of E, whose size is the residual):
// the errors of Y1 = Z V_f and Y2 = Z^T U_f fall with err_k. The threshold
// decisions, the residual and err_k are the FP32 ones.
//
// Layout: workgroup of 4 waves, tile TM rows x 256 columns, processed in
// rounds of four 16-row blocks (wave w takes rows i0 + 16w .. i0 + 16w + 15 of
// each round). Phase A: the lane owns columns 4l..4l+3, loads mx_batch(K) rows
// at a time (the next batch in flight), and writes BF16 E row-major into its
// wave's LDS block (row pitch 260 BF16: the pad spreads the row reads over the
// banks); the wave also puts its block's rows of U_f (BF16) into a shared
// t-major table. After a workgroup barrier, phase B: E V_f of the wave's own
// 16 rows (eight v_mfma_f32_16x16x32_bf16 over the 32-column blocks, A read
// from the wave's block, 8 consecutive columns per lane), and E^T U_f of the
// wave's own 64 columns over the round's 64 rows (sixteen
// v_mfma_f32_16x16x16_bf16: 4 column blocks x the 4 waves' row blocks, E read
// from every wave's block, 4 rows of one column per lane), accumulated in
// registers over the rounds; a second barrier frees the blocks for the next
// round. MFMA lane layouts (16 x 16 output, k-width 8 or 4 per lane): A row
// l%16, k = 8(l/16)+q (or 4(l/16)+q); B column l%16, same k; C column l%16,
// rows 4(l/16)+r. Partials are written in the FP32 pass's layout, so the
// gather is shared.

#include "launch.hpp"
#include "wave.hpp"

namespace rpca {
namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef short i16x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

constexpr int MX_RB = 16;                 // rows per wave block (MFMA M)
constexpr int MX_PITCH = STREAM_TN + 4;   // BF16 per LDS row
// U_f rows of a round in LDS: one line per column t < K of U_f, 64 rows + pad
// per line (136 bytes, a multiple of 8)
constexpr int MX_UROWS = MX_RB * STREAM_WAVES;
constexpr int MX_UPITCH = MX_UROWS + 4;
// rows per batch of loads in phase A: 4, or 2 from K = 8 on, where the
// registers of two batches in flight would cost a wave per SIMD
constexpr int mx_batch(int K) { return K >= 8 ? 2 : 4; }

__device__ inline uint32_t pack2(float a, float b) {
    const __bf16 ha = static_cast<__bf16>(a), hb = static_cast<__bf16>(b);
    return (uint32_t)__builtin_bit_cast(uint16_t, ha) | ((uint32_t)__builtin_bit_cast(uint16_t, hb) << 16);
}

__device__ inline __bf16 to_bf16(float x) { return static_cast<__bf16>(x); }
__device__ inline uint16_t bf16_bits(float x) { return __builtin_bit_cast(uint16_t, static_cast<__bf16>(x)); }

// NBT rows x 4 columns of D for one lane (zeros outside the matrix).
// FULL: the tile's 256 columns are inside D and rows are 16-byte aligned, so
// only the (wave-uniform) row bound is checked.
template <int NBT, bool FULL, bool NT>
__device__ inline void mx_load_batch(const float* __restrict__ D, int64_t ldd, int i0, int i_hi, int jb, int nvalid,
                                     float (&d)[NBT][4]) {
#pragma unroll
    for (int b = 0; b < NBT; ++b) {
        const int i = i0 + b;
        const float* p = D + (size_t)i * ldd + jb;
        if constexpr (FULL) {
            if (i < i_hi) {
                const float4 v = load_d<NT>(reinterpret_cast<const float4*>(p));
                d[b][0] = v.x; d[b][1] = v.y; d[b][2] = v.z; d[b][3] = v.w;
            } else {
#pragma unroll
                for (int s = 0; s < 4; ++s) d[b][s] = 0.f;
            }
        } else {
#pragma unroll
            for (int s = 0; s < 4; ++s) d[b][s] = (i < i_hi && s < nvalid) ? load_d<NT>(p + s) : 0.f;
        }
    }
}

// Threshold and residual of one batch; E in BF16 into the wave's LDS block.
// CHECK: some rows of the batch may lie past i_hi (wave-uniform choice); a
// batch inside the tile loads its row operands without per-row conditions.
// Rows past i_hi give E = 0.
template <int K, int NBT, bool REBUILD, bool CHECK>
__device__ inline void mx_compute_batch(const float (&d)[NBT][4], const float* __restrict__ AL, int i0, int i_hi,
                                        int r_local, float zeta, const float (&bl)[4][K], uint16_t* zl, int lane,
                                        float& rs, float& amax) {
#pragma unroll
    for (int b = 0; b < NBT; ++b) {
        const int i = i0 + b;
        float al[K];
#pragma unroll
        for (int t = 0; t < K; ++t) al[t] = (REBUILD && (!CHECK || i < i_hi)) ? AL[(size_t)i * K + t] : 0.f;
        float ev[4];
#pragma unroll
        for (int s = 0; s < 4; ++s) {
            const float dv = d[b][s];
            float x = dv;
            if constexpr (REBUILD) {
#pragma unroll
                for (int t = 0; t < K; ++t) x = fmaf(-al[t], bl[s][t], x);
            } else {
                amax = fmaxf(amax, fabsf(x));
            }
            const bool big = fabsf(x) > zeta;   // S_ij = x
            const float e = big ? 0.f : x;      // entry of E = D - L - S
            rs = fmaf(e, e, rs);
            ev[s] = e;
        }
        uint2 w;
        w.x = pack2(ev[0], ev[1]);
        w.y = pack2(ev[2], ev[3]);
        *reinterpret_cast<uint2*>(zl + (r_local + b) * MX_PITCH + 4 * lane) = w;
    }
}

template <int K, bool REBUILD, bool FULL>
__device__ inline void mx_tile(const float* __restrict__ D, const float* __restrict__ AL,
                               const float* __restrict__ Uf, float* __restrict__ P1, const StreamGeom& g, float zeta,
                               int ct, int i_lo, int i_hi, int wave, int lane, int jb, int nvalid,
                               const float (&bl)[4][K], f32x4 (&acc2)[4], const bf16x8* vl,
                               uint16_t (*zbuf)[MX_RB * MX_PITCH], uint16_t* ul, double& res, float& amax) {
    const int lr = lane & 15, lg = lane >> 4;
    const int tl = lr < K ? lr : K - 1;   // A lines of Y2: lanes with t >= K give zeros
    const bf16x8 zero8 = {};
    const i16x4 zero4 = {};
    constexpr int NBT = mx_batch(K);
    uint16_t* zl = zbuf[wave];
    float ba[NBT][4], bb[NBT][4];
    // rounds of four 16-row blocks; every wave takes part in every round (a
    // block past i_hi is all zeros), so the barriers are uniform
    const int nblk = i_hi > i_lo ? (i_hi - i_lo + MX_RB - 1) / MX_RB : 0;
    const int rounds = (nblk + STREAM_WAVES - 1) / STREAM_WAVES;
    int i0 = i_lo + MX_RB * wave;
    if (rounds > 0) mx_load_batch<NBT, FULL, (K <= D_LOADS_NT_KMAX)>(D, g.ldd, i0, i_hi, jb, nvalid, ba);
    for (int rd = 0; rd < rounds; ++rd, i0 += MX_RB * STREAM_WAVES) {
        float rs = 0.f;
        // phase A: batches of NBT rows in two register buffers; the loads
        // of the next batch (or of the next block's first batch) are in flight
        // while one is computed. Rows at or past i_hi load as zeros.
        const int i_next = i0 + MX_RB * STREAM_WAVES;
#pragma unroll 1
        for (int bt = 0; bt < MX_RB / NBT; bt += 2) {
            mx_load_batch<NBT, FULL, (K <= D_LOADS_NT_KMAX)>(D, g.ldd, i0 + NBT * (bt + 1), i_hi, jb, nvalid, bb);
            if (i0 + NBT * (bt + 1) <= i_hi)
                mx_compute_batch<K, NBT, REBUILD, false>(ba, AL, i0 + NBT * bt, i_hi, NBT * bt, zeta, bl, zl, lane,
                                                         rs, amax);
            else
                mx_compute_batch<K, NBT, REBUILD, true>(ba, AL, i0 + NBT * bt, i_hi, NBT * bt, zeta, bl, zl, lane,
                                                        rs, amax);
            const int inx = (bt + 2 < MX_RB / NBT) ? i0 + NBT * (bt + 2) : i_next;
            mx_load_batch<NBT, FULL, (K <= D_LOADS_NT_KMAX)>(D, g.ldd, inx, i_hi, jb, nvalid, ba);
            if (i0 + NBT * (bt + 2) <= i_hi)
                mx_compute_batch<K, NBT, REBUILD, false>(bb, AL, i0 + NBT * (bt + 1), i_hi, NBT * (bt + 1), zeta,
                                                         bl, zl, lane, rs, amax);
            else
                mx_compute_batch<K, NBT, REBUILD, true>(bb, AL, i0 + NBT * (bt + 1), i_hi, NBT * (bt + 1), zeta, bl,
                                                        zl, lane, rs, amax);
        }
        res += static_cast<double>(rs);
        // the block's rows of U_f (BF16) into the round's table, t-major
        for (int e = lane; e < MX_RB * K; e += WAVE) {
            const int r = e / K, t = e - (e / K) * K;
            const int i = i0 + r;
            ul[t * MX_UPITCH + MX_RB * wave + r] = bf16_bits(i < i_hi ? Uf[(size_t)i * K + t] : 0.f);
        }
        __syncthreads();   // every wave's E block and U_f rows of the round are in LDS

        // phase B, Y1 = E V_f of the wave's own block: rows i0 + lr, columns 32kb + 8lg + q
        if (i0 < i_hi) {
            f32x4 a1 = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
            for (int kb = 0; kb < STREAM_TN / 32; ++kb) {
                const uint16_t* src = zl + lr * MX_PITCH + 32 * kb + 8 * lg;
                const uint2 w0 = *reinterpret_cast<const uint2*>(src);
                const uint2 w1 = *reinterpret_cast<const uint2*>(src + 4);
                const uint32_t wv[4] = {w0.x, w0.y, w1.x, w1.y};
                bf16x8 A = __builtin_bit_cast(bf16x8, wv);
                const bf16x8 B = lr < K ? vl[(kb * 4 + lg) * K + lr] : zero8;
                a1 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(A, B, a1, 0, 0, 0);
            }
            if (lr < K) {
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int i = i0 + 4 * lg + r;
                    if (i < i_hi) P1[((size_t)ct * g.m + i) * K + lr] = a1[r];
                }
            }
        }
        // phase B, Y2 = E^T U_f of the wave's own 64 columns over the round's
        // 64 rows: C[t][col] += U^T (rows of block b) E (rows of block b, col)
        // A: t = lr, rows 4lg + q of block b; B: column 64 wave + 16 st + lr, same rows
#pragma unroll
        for (int b = 0; b < STREAM_WAVES; ++b) {
            i16x4 A = *reinterpret_cast<const i16x4*>(ul + tl * MX_UPITCH + MX_RB * b + 4 * lg);
            if (lr >= K) A = zero4;
            const uint16_t* zb = zbuf[b] + (4 * lg) * MX_PITCH + 64 * wave + lr;
#pragma unroll
            for (int st = 0; st < 4; ++st) {
                i16x4 B;
#pragma unroll
                for (int q = 0; q < 4; ++q) B[q] = (short)zb[q * MX_PITCH + 16 * st];
                acc2[st] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(A, B, acc2[st], 0, 0, 0);
            }
        }
        __syncthreads();   // the blocks and the table are free for the next round
    }
}

template <int K, bool REBUILD>
__global__ __launch_bounds__(STREAM_THREADS) void k_stream_mx(
    const float* __restrict__ D, const float* __restrict__ AL, const float* __restrict__ BL,
    const float* __restrict__ Uf, const float* __restrict__ Vf, float* __restrict__ P1, float* __restrict__ P2,
    double* __restrict__ resid, Ctrl* __restrict__ ctrl, StreamGeom g) {
    static_assert(K <= 16, "MFMA N = 16 holds up to 16 columns");
    {   // instance blockIdx.y of a batched launch (slab 0: a single instance)
        const int64_t off = (int64_t)blockIdx.y * g.slab;
        D = moved(D, off);
        AL = moved(AL, off);
        BL = moved(BL, off);
        Uf = moved(Uf, off);
        Vf = moved(Vf, off);
        P1 = moved(P1, off);
        P2 = moved(P2, off);
        resid = moved(resid, off);
        ctrl = moved(ctrl, off);
    }
    if (!body_runs(ctrl, g.body)) return;
    const float zeta = static_cast<float>(ctrl->zeta);
    const int lane = threadIdx.x & (WAVE - 1);
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x / WAVE);
    // (numbering the tiles per XCD, as the FP32 pass does, measured 2-5 %
    // slower for this pass at r = 5 and r = 10)
    const int tile = blockIdx.x;
    const int ct = tile % g.n_ct;
    const int rt = tile / g.n_ct;
    const int c0 = ct * STREAM_TN;
    const int jb = c0 + lane * 4;
    const int nvalid = min(max(g.n - jb, 0), 4);
    const int i_lo = rt * g.TM;
    const int i_hi = min(g.m, i_lo + g.TM);

    // E blocks; afterwards, scratch of pass_finishes_update
    __shared__ __align__(16) uint16_t zbuf[STREAM_WAVES][MX_RB * MX_PITCH];
    static_assert(sizeof(zbuf) >= FINISH_LDS<K, STREAM_THREADS>() * sizeof(double), "scratch of the closing sums");
    __shared__ __align__(8) uint16_t ul[K * MX_UPITCH];
    __shared__ double red[STREAM_WAVES];
    // B operands of Y1 in LDS: for (32-column block kb, k group lg, column t
    // < K) the 8 BF16 values V_f[c0 + 32kb + 8lg + q][t]
    __shared__ bf16x8 vl[(STREAM_TN / 32) * 4 * K];
    for (int e = threadIdx.x; e < (STREAM_TN / 32) * 4 * K; e += STREAM_THREADS) {
        const int t = e % K, grp = (e / K) % 4, kb = e / (4 * K);
        bf16x8 v;
#pragma unroll
        for (int q = 0; q < 8; ++q) {
            const int j = c0 + 32 * kb + 8 * grp + q;
            v[q] = to_bf16(j < g.n ? Vf[(size_t)j * K + t] : 0.f);
        }
        vl[e] = v;
    }
    __syncthreads();

    float bl[4][K];
#pragma unroll
    for (int s = 0; s < 4; ++s)
#pragma unroll
        for (int t = 0; t < K; ++t) bl[s][t] = (REBUILD && s < nvalid) ? BL[(size_t)(jb + s) * K + t] : 0.f;
    f32x4 acc2[4];
#pragma unroll
    for (int st = 0; st < 4; ++st) acc2[st] = f32x4{0.f, 0.f, 0.f, 0.f};
    double res = 0.0;
    float amax = 0.f;
    const bool full = g.vec_ok && c0 + STREAM_TN <= g.n;   // uniform per workgroup
    if (full)
        mx_tile<K, REBUILD, true>(D, AL, Uf, P1, g, zeta, ct, i_lo, i_hi, wave, lane, jb, nvalid, bl, acc2, vl, zbuf,
                                  ul, res, amax);
    else
        mx_tile<K, REBUILD, false>(D, AL, Uf, P1, g, zeta, ct, i_lo, i_hi, wave, lane, jb, nvalid, bl, acc2, vl,
                                   zbuf, ul, res, amax);

    // Y2 partial of the tile: the wave's 64 columns, t = 4 (lane / 16) + r
    {
        const int lr = lane & 15, lg = lane >> 4;
#pragma unroll
        for (int st = 0; st < 4; ++st) {
            const int col = c0 + 64 * wave + 16 * st + lr;
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int t = 4 * lg + r;
                if (t < K && col < g.n) P2[((size_t)rt * g.n + col) * K + t] = acc2[st][r];
            }
        }
    }
    const double rtot = block_sum_256(res, red);
    if (threadIdx.x == 0) resid[tile] = rtot;
    if constexpr (!REBUILD) {
        double v = static_cast<double>(amax);
        for (int off = 32; off > 0; off >>= 1) v = fmax(v, __shfl_xor(v, off, WAVE));
        if (lane == 0) red[wave] = v;
        __syncthreads();
        if (threadIdx.x == 0) {
            double mx = red[0];
            for (int w = 1; w < STREAM_WAVES; ++w) mx = fmax(mx, red[w]);
            resid[gridDim.x + tile] = mx;
        }
    }
    pass_finishes_update<K, STREAM_THREADS>(ctrl, g, (int64_t)blockIdx.y * g.slab, reinterpret_cast<double*>(&zbuf[0][0]));
}

template <bool REBUILD>
hipError_t mx_dispatch(const StreamArgs& a, int K, hipStream_t s) {
    const dim3 grid((unsigned)(a.n_ct * a.n_rt), a.batch > 1 ? (unsigned)a.batch : 1u), block(STREAM_THREADS);
    StreamGeom geom;
    geom.slab = a.batch > 1 ? a.slab : 0;
    geom.ldd = a.ldd;
    geom.m = a.m;
    geom.n = a.n;
    geom.TM = a.TM;
    geom.n_ct = a.n_ct;
    geom.n_rt = a.n_rt;
    geom.vec_ok = a.vec_ok;
    geom.body = a.body;
    geom.post_gpart = a.post_gpart;
    geom.post_small = a.post_small;
    geom.post_gU = a.post_gU;
    geom.post_gV = a.post_gV;
    switch (K) {
#define RPCA_CASE(KK)                                                                                        \
    case KK:                                                                                                 \
        hipLaunchKernelGGL((k_stream_mx<KK, REBUILD>), grid, block, 0, s, static_cast<const float*>(a.D),    \
                           static_cast<const float*>(a.AL), static_cast<const float*>(a.BL),                 \
                           static_cast<const float*>(a.Uf), static_cast<const float*>(a.Vf),                 \
                           static_cast<float*>(a.P1), static_cast<float*>(a.P2), a.resid, a.ctrl, geom);     \
        break;
        RPCA_CASE(1) RPCA_CASE(2) RPCA_CASE(3) RPCA_CASE(4) RPCA_CASE(5) RPCA_CASE(6)
        RPCA_CASE(7) RPCA_CASE(8) RPCA_CASE(9) RPCA_CASE(10) RPCA_CASE(11) RPCA_CASE(12)
        RPCA_CASE(13) RPCA_CASE(14) RPCA_CASE(15) RPCA_CASE(16)
#undef RPCA_CASE
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

template <bool REBUILD>
int mx_occupancy_t(int K) {
    int n = 0;
    hipError_t e = hipErrorInvalidValue;
    switch (K) {
#define RPCA_CASE(KK)                                                                                   \
    case KK:                                                                                            \
        e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k_stream_mx<KK, REBUILD>, STREAM_THREADS, 0); \
        break;
        RPCA_CASE(1) RPCA_CASE(2) RPCA_CASE(3) RPCA_CASE(4) RPCA_CASE(5) RPCA_CASE(6)
        RPCA_CASE(7) RPCA_CASE(8) RPCA_CASE(9) RPCA_CASE(10) RPCA_CASE(11) RPCA_CASE(12)
        RPCA_CASE(13) RPCA_CASE(14) RPCA_CASE(15) RPCA_CASE(16)
#undef RPCA_CASE
        default: break;
    }
    return (e == hipSuccess && n > 0) ? n : 1;
}

}  // namespace

int stream_mx_occupancy(int K, bool rebuild) {
    return rebuild ? mx_occupancy_t<true>(K) : mx_occupancy_t<false>(K);
}

hipError_t launch_stream_mx(const StreamArgs& a, int K, bool rebuild, hipStream_t s) {
    return rebuild ? mx_dispatch<true>(a, K, s) : mx_dispatch<false>(a, K, s);
}

}  // namespace rpca
