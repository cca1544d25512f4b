// kernels_mfma.hip -- dense J times a block of R restarts on the matrix cores.
//
// With R restarts the DOCH matvec becomes Z = J U, a dense (n x n) by (n x R)
// product with reuse, which belongs on MFMA.  The iteration runs on
// u = sqrt(beta) x, for which eq:FPE reads u <- cbrt(J u + alpha u) (beta
// drops out exactly), so the iterate stays O(sqrt(alpha + lambda)) and is
// representable in BF16 and in FP8 (e4m3, largest finite 448).
//
// J sits in a BF16 copy, or an FP8 copy with one FP32 scale per row
// (J_ij ~ s_i q_ij, s_i = max_j |J_ij| / 448).  The restart block sits as an
// FP32 master (n x R) plus a low-precision transposed copy (R x n) that
// feeds the next product.  In FP8 that copy carries one FP32 scale per
// restart, c_j, with |u_ij| <= 448 c_j: exact at the start (column maximum)
// and carried forward by the bound |u'| = |cbrt(z + alpha u)| <=
// cbrt((rho_q + alpha) M) for |u| <= M, where rho_q is the largest absolute
// row sum of the quantised J.  The bound tends to sqrt(rho_q + alpha), so
// large starting points (u = sqrt(beta) x is large when beta is) never reach
// the format's overflow, and later steps keep its full relative precision.
//
// Four shapes of one iteration (chosen per problem by the caller or by
// timing them):
//   fused      one launch per iteration; a workgroup owns a 64 x 64 tile of
//              Z over the whole k range and updates it in place;
//   resident   the fused tile body for every iteration in one cooperative
//              launch, grid barriers between iterations;
//   split      128 x bn tiles over 1..8 splits of the k range into FP32
//              partial tiles, then an update kernel that adds them;
//   held       one cooperative launch whose workgroups keep a 128-row k
//              slice of J in LDS for the whole run: split products, a grid
//              barrier, the update, a grid barrier per iteration.
// The first three stage the k range through LDS in stages of whole cache
// lines; every shape ends an iteration the same way: the update (z + alpha
// u in FP64, its cube root in FP32, the precision u is stored in), both
// copies stored, the restart's FP64 partial sums per row tile, and the
// iteration closed for every restart (H, r, freezing at r < eps) while the
// next one runs.
#include "device_common.h"
#include "ising_internal.h"

namespace doch {

namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x16 __attribute__((ext_vector_type(16)));

constexpr int MT = 256;        // threads per workgroup

template <int PREC> struct Prec;
template <> struct Prec<0> {   // BF16
    using T = __bf16;
};
template <> struct Prec<1> {   // FP8 e4m3 (OCP)
    using T = uint8_t;
};

constexpr float kFp8Max = 448.0f;
// margin on the carried bound: FP32 accumulation of the product (relative
// error below n 2^-24 <= 2^-8 for n <= 65536) and rounding of the update
constexpr double kBoundSlack = 1.01;

__device__ __forceinline__ uint8_t to_fp8(float f) {
    // v_cvt_pk_fp8_f32 rounds to nearest even; the operands are scaled into
    // range, the clamp only guards the boundary
    f = fminf(fmaxf(f, -kFp8Max), kFp8Max);
    return static_cast<uint8_t>(__builtin_amdgcn_cvt_pk_fp8_f32(f, 0.0f, 0, false) & 0xff);
}

// OCP e4m3 code -> value: bias 7, 3 mantissa bits, subnormals at exponent 0
__device__ __forceinline__ double fp8_value(uint8_t q) {
    const int e = (q >> 3) & 15, m = q & 7;
    const double mag = e == 0 ? ldexp(static_cast<double>(m), -9) : ldexp(1.0 + m / 8.0, e - 7);
    return (q & 0x80) ? -mag : mag;
}

// carried bound of the next iterate's magnitude, as a restart scale
__device__ __forceinline__ float next_colscale(float c_old, double rho_q, double alpha) {
    const double m_old = dmul(static_cast<double>(kFp8Max), static_cast<double>(c_old));
    const double m_new = dmul(kBoundSlack, cbrt(dmul(dadd(dmul(kBoundSlack, rho_q), alpha), m_old)));
    return static_cast<float>(dmul(ddiv(m_new, static_cast<double>(kFp8Max)), kBoundSlack));
}

template <int PREC>
__device__ __forceinline__ typename Prec<PREC>::T to_lowp(float f) {
    if constexpr (PREC == 0) return static_cast<__bf16>(f);
    else return to_fp8(f);
}

// Finish iteration kk of restart c from its four FP64 sums over all rows
// (u^4, u^2, u z, (du)^2): H, r, the log and the state (eq:Hamilton in
// u = sqrt(beta) x, Remark S2).
__device__ __forceinline__ void lowp_close_restart(const double (&S)[4], int c, int R, int64_t kk, double alpha,
                                                   double beta, double eps, double* __restrict__ log,
                                                   RestartState* __restrict__ state, int done = -1) {
    if (c >= R || (done < 0 ? state[c].done : done)) return;
    // H(x) = H_u / beta with x = u / sqrt(beta); r is scale free
    const double Hu = dsub(dsub(dmul(0.25, S[0]), dmul(ddiv(alpha, 2.0), S[1])), dmul(0.5, S[2]));
    const double H = ddiv(Hu, beta);
    const double r = S[1] == 0.0 ? 0.0 : ddiv(sqrt(S[3]), sqrt(S[1]));
    log[(static_cast<size_t>(kk) * R + c) * 2] = H;
    log[(static_cast<size_t>(kk) * R + c) * 2 + 1] = r;
    RestartState& st = state[c];
    st.iters_done = kk + 1;
    st.H_last = H;
    st.r_last = r;
    if (!isfinite(H) || !isfinite(r)) {
        st.nonfinite = 1;
        st.done = 1;
    } else if (eps > 0.0 && r < eps) {
        st.converged = 1;
        st.done = 1;
    }
}

// Close iteration kk of the 64 restarts of column block cb: add the row
// tiles' partial sums in tile order (0, 1, ..., tiles - 1), then finish each
// restart.  red: 64 x 4 doubles of LDS.
__device__ void lowp_close(const double* __restrict__ P, int tiles, int Rp, int cb, int R, int64_t kk,
                           double alpha, double beta, double eps, double* __restrict__ log,
                           RestartState* __restrict__ state, double (*red)[4]) {
    const int tid = threadIdx.x;
    const int col0 = cb * 64;
    {
        const int cl = tid & 63, q = tid >> 6;
        red[cl][q] = column_partial_sum<4>(P, Rp, col0 + cl, q, tiles);
    }
    __syncthreads();
    if (tid < 64) {
        const double S[4] = {red[tid][0], red[tid][1], red[tid][2], red[tid][3]};
        lowp_close_restart(S, col0 + tid, R, kk, alpha, beta, eps, log, state);
    }
}


// ---- the product: split-k partial tiles --------------------------------
//
// P[s] = J[:, K_s] U^T[K_s, :] for split s of the k range, as FP32 partial
// tiles (np x Rp, row-major).  A workgroup owns a 128 x BN tile of one
// split; its four wavefronts split the tile 2 x 2 and each accumulates its
// 64 x BN/2 sub-tile as 2 x BN/64 independent 32 x 32 MFMA blocks over the
// whole k range of the split (no reduction inside the workgroup).  The k
// range streams in stages of SB bytes per row: every row of J and of the
// restart copy that the tile needs is loaded as whole cache lines into
// registers DEPTH stages ahead, written to one of two LDS buffers, and read
// back as MFMA fragments -- one barrier per stage.  Stages of SB = 256 bytes
// per row take about 136 KB of LDS at BN = 128 (one workgroup per compute
// unit); SB = 128 halves that, so two workgroups can share one.
//
// Fragment layout: lane l takes row l % 32 of its 32-row block and half
// l / 32 of the k-step's bytes (16 bytes of BF16 for the 32 x 32 x 16 MFMA,
// 32 bytes of FP8 for the 32 x 32 x 64 one).  Both operands are read the
// same way, so the products pair k with k whatever order the matrix core
// assigns to the bytes inside a fragment.
constexpr int kTileM = 128;                    // rows of J per product tile

typedef int i32x8 __attribute__((ext_vector_type(8)));

// bytes of k per MFMA step, and the step itself on two LDS fragments
template <int PREC> struct Mfma;
template <> struct Mfma<0> {
    static constexpr int kBytes = 32;         // 32 x 32 x 16 BF16
    typedef bf16x8 frag;
    static __device__ __forceinline__ frag load(const char* p) { return *reinterpret_cast<const bf16x8*>(p); }
    static __device__ __forceinline__ f32x16 step(frag a, frag b, f32x16 c) {
        return __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, c, 0, 0, 0);
    }
};
template <> struct Mfma<1> {
    static constexpr int kBytes = 64;         // 32 x 32 x 64 FP8 (e4m3 both operands, no block scales)
    typedef i32x8 frag;
    static __device__ __forceinline__ frag load(const char* p) {
        const i32x4 lo = *reinterpret_cast<const i32x4*>(p);
        const i32x4 hi = *reinterpret_cast<const i32x4*>(p + 16);
        return __builtin_shufflevector(lo, hi, 0, 1, 2, 3, 4, 5, 6, 7);
    }
    static __device__ __forceinline__ f32x16 step(frag a, frag b, f32x16 c) {
        // format codes 0/0: e4m3 x e4m3; zero scale operands select the
        // unscaled instruction
        return __builtin_amdgcn_mfma_scale_f32_32x32x64_f8f6f4(a, b, c, 0, 0, 0, 0, 0, 0);
    }
};

__device__ __forceinline__ __amdgpu_buffer_rsrc_t slab_rsrc(const void* base, uint32_t bytes) {
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(base), static_cast<short>(0),
                                             static_cast<int>(bytes), 0x00020000);
}

template <int PREC, int BN, int SB, int DEPTH>
__device__ __forceinline__ void lowp_gemm_tile(int np, int Rp, int S, int R,
                                                       const typename Prec<PREC>::T* __restrict__ Jq,
                                                       const typename Prec<PREC>::T* __restrict__ Ub,
                                                       float* __restrict__ P, int64_t k, double alpha,
                                                       double beta, double eps,
                                                       const double* __restrict__ partials_prev,
                                                       double* __restrict__ log,
                                                       RestartState* __restrict__ state) {
    using T = typename Prec<PREC>::T;
    using M = Mfma<PREC>;
    constexpr int ROWS = kTileM + BN;          // staged rows: J, then restarts
    constexpr int TN = BN / 64;                // 32-column blocks per wavefront
    constexpr int kSrow = SB + 16;             // LDS row pitch: 16-row groups hit distinct banks
    constexpr int CPR = SB / 16;               // 16-byte chunks per row per stage
    constexpr int RPU = MT / CPR;              // rows one load instruction of the workgroup covers
    constexpr int LJ = kTileM / RPU, LU = BN / RPU;   // 16-byte loads per thread per stage
    constexpr int FB = M::kBytes / 2;          // fragment bytes per lane
    __shared__ __attribute__((aligned(16))) char lds[2 * ROWS * kSrow];

    // tile of this workgroup: consecutive logical tiles share an XCD (round-
    // robin dispatch), so the column tiles of one (row tile, split) -- which
    // read the same slab of J -- meet in one L2
    const int tn = Rp / BN;
    const int G = (np / kTileM) * tn * S;
    const int b = blockIdx.x;
    // the Rp / 64 workgroups after the product tiles close the previous
    // iteration, whose partial sums the previous update wrote; with stages
    // of 128 bytes a workgroup takes little enough LDS for one of them to
    // share a compute unit with a product tile
    if (b >= G) {
        if (k > 0)
            lowp_close(partials_prev, np / 64, Rp, b - G, R, k - 1, alpha, beta, eps, log, state,
                       reinterpret_cast<double(*)[4]>(lds));
        return;
    }
    int L = (G & 7) == 0 ? (b & 7) * (G >> 3) + (b >> 3) : b;
    const int nt = L % tn;
    L /= tn;
    const int s = L % S;
    const int mt = L / S;
    const int row0 = mt * kTileM, col0 = nt * BN;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wr = wave >> 1, wc = wave & 1;

    // a tile whose restarts have all stopped is not needed
    const int cc = col0 + tid;
    const bool live = tid < BN && cc < R && !state[cc].done;
    if (!__syncthreads_or(live)) return;

    const uint32_t rowb = static_cast<uint32_t>(np) * sizeof(T);   // bytes per row of J and of the copy
    const uint32_t kw = rowb / S;                                    // k bytes of this split
    const int nst = static_cast<int>(kw / SB);
    const __amdgpu_buffer_rsrc_t rJ =
        slab_rsrc(reinterpret_cast<const char*>(Jq) + static_cast<size_t>(row0) * rowb + static_cast<size_t>(s) * kw,
                  kTileM * rowb);
    const __amdgpu_buffer_rsrc_t rU =
        slab_rsrc(reinterpret_cast<const char*>(Ub) + static_cast<size_t>(col0) * rowb + static_cast<size_t>(s) * kw,
                  BN * rowb);
    // chunk (row RPU u + tid / CPR, bytes 16 (tid % CPR)) of a stage: CPR
    // lanes read one row's stage as whole cache lines
    const uint32_t voff = (tid / CPR) * rowb + (tid % CPR) * 16;
    const int soff = (tid / CPR) * kSrow + (tid % CPR) * 16;
    i32x4 ring[DEPTH][LJ + LU];
    auto fetch = [&](i32x4 (&r)[LJ + LU], int st) {
        const uint32_t o = voff + static_cast<uint32_t>(st) * SB;
#pragma unroll
        for (int u = 0; u < LJ; ++u) r[u] = __builtin_amdgcn_raw_buffer_load_b128(rJ, o, u * RPU * rowb, 0);
#pragma unroll
        for (int u = 0; u < LU; ++u) r[LJ + u] = __builtin_amdgcn_raw_buffer_load_b128(rU, o, u * RPU * rowb, 0);
    };
    // every split holds at least DEPTH stages (lowp_shape_valid)
#pragma unroll
    for (int p = 0; p < DEPTH; ++p) fetch(ring[p], p);

    f32x16 acc[2][TN];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < TN; ++j) acc[i][j] = f32x16{};
    const int fa = (wr * 64 + (lane & 31)) * kSrow + (lane >> 5) * FB;
    const int fb = (kTileM + wc * (BN / 2) + (lane & 31)) * kSrow + (lane >> 5) * FB;
    // stage st: its registers to LDS buffer st % 2, the refetch DEPTH stages
    // ahead into the same registers, one barrier, the MFMA steps
    auto stage = [&](i32x4 (&r)[LJ + LU], int st, bool refetch) {
        char* buf = lds + (st & 1) * ROWS * kSrow;
#pragma unroll
        for (int u = 0; u < LJ + LU; ++u) *reinterpret_cast<i32x4*>(buf + soff + u * RPU * kSrow) = r[u];
        if (refetch) fetch(r, st + DEPTH);
        __syncthreads();
#pragma unroll
        for (int ks = 0; ks < SB / M::kBytes; ++ks) {
            typename M::frag a[2], bb[TN];
#pragma unroll
            for (int i = 0; i < 2; ++i) a[i] = M::load(buf + fa + i * 32 * kSrow + ks * M::kBytes);
#pragma unroll
            for (int j = 0; j < TN; ++j) bb[j] = M::load(buf + fb + j * 32 * kSrow + ks * M::kBytes);
#pragma unroll
            for (int i = 0; i < 2; ++i)
#pragma unroll
                for (int j = 0; j < TN; ++j) acc[i][j] = M::step(a[i], bb[j], acc[i][j]);
        }
    };
    // steady state: every stage refetches, so the loads of the next DEPTH - 1
    // stages stay in flight across each wait; the last stages (at most
    // 2 DEPTH - 1) follow with the refetch where one is left
    int s0 = 0;
    for (; s0 + 2 * DEPTH <= nst; s0 += DEPTH) {
#pragma unroll
        for (int p = 0; p < DEPTH; ++p) stage(ring[p], s0 + p, true);
    }
#pragma unroll
    for (int q = 0; q < 2 * DEPTH - 1; ++q) {
        const int st = s0 + q;
        if (st < nst) stage(ring[q % DEPTH], st, st + DEPTH < nst);
    }
    // lane holds column l % 32 and rows 8 (v / 4) + 4 (l / 32) + v % 4 of
    // each 32 x 32 block
    float* Ps = P + static_cast<size_t>(s) * np * Rp;
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < TN; ++j)
#pragma unroll
            for (int v = 0; v < 16; ++v) {
                const int r = row0 + wr * 64 + i * 32 + 8 * (v >> 2) + 4 * (lane >> 5) + (v & 3);
                const int c = col0 + wc * (BN / 2) + j * 32 + (lane & 31);
                Ps[static_cast<size_t>(r) * Rp + c] = acc[i][j][v];
            }
}


#define DOCH_LOWP_GEMM_PARAMS                                                                              \
    int np, int Rp, int S, int R, const typename Prec<PREC>::T *__restrict__ Jq,                          \
        const typename Prec<PREC>::T *__restrict__ Ub, float *__restrict__ P, int64_t k, double alpha,    \
        double beta, double eps, const double *__restrict__ partials_prev, double *__restrict__ log,      \
        RestartState *__restrict__ state
#define DOCH_LOWP_GEMM_ARGS np, Rp, S, R, Jq, Ub, P, k, alpha, beta, eps, partials_prev, log, state

// 256-byte stages: one workgroup per compute unit, registers unconstrained
template <int PREC, int BN, int DEPTH>
__global__ __launch_bounds__(MT) void lowp_gemm_kernel(DOCH_LOWP_GEMM_PARAMS) {
    lowp_gemm_tile<PREC, BN, 256, DEPTH>(DOCH_LOWP_GEMM_ARGS);
}

// 128-byte stages: registers kept to two wavefronts per SIMD, so a second
// workgroup (a closing one, or a product tile when there are more tiles
// than compute units) fits beside each product tile
template <int PREC, int BN, int DEPTH>
__global__ __launch_bounds__(MT) __attribute__((amdgpu_waves_per_eu(2))) void lowp_gemm2_kernel(
    DOCH_LOWP_GEMM_PARAMS) {
    lowp_gemm_tile<PREC, BN, 128, DEPTH>(DOCH_LOWP_GEMM_ARGS);
}
#undef DOCH_LOWP_GEMM_PARAMS
#undef DOCH_LOWP_GEMM_ARGS

// ---- the fused iteration: one 64 x 64 tile per workgroup, whole k range --
//
// The product and the update with no partial tiles in memory: a workgroup
// owns 64 rows x 64 restarts; each of its four wavefronts accumulates the
// whole tile as 2 x 2 independent 32 x 32 MFMA blocks over every fourth MFMA
// step of each 256-byte stage, the four partial tiles meet in LDS
// (wavefront w keeps sub-tile w, summed over the wavefronts in order), and
// the epilogue is the update's.  The tiles also close the previous
// iteration (FusedClose): no workgroup of its own does it, because one
// sharing a compute unit with a tile slowed that tile by 2 us and with it
// the whole iteration.  It runs either as one launch per iteration
// (lowp_fused_kernel; registers capped at two wavefronts per SIMD, which
// measured 24.0 against 24.6 us per BF16 iteration without the cap) or
// resident for the whole run (lowp_resident_kernel).

constexpr int kFusedStage = 256;                      // k bytes per row per stage
constexpr int kFusedSrow = kFusedStage + 16;          // LDS row pitch
// two stage buffers (J rows, then restart rows; 64 rows each), reused for
// the four wavefronts' partial tiles ([wave][sub-tile][v][lane] floats) and
// then for the transposed low-precision copy
constexpr int kFusedStageLds = 2 * 2 * 64 * kFusedSrow > 4 * 4 * 16 * 64 * 4 ? 2 * 2 * 64 * kFusedSrow
                                                                               : 4 * 4 * 16 * 64 * 4;
struct FusedLds {
    __attribute__((aligned(16))) char stage[kFusedStageLds];
    double red[2][64][4];
    double close_s[64][4];      // sums of the restarts this tile closes
    double close_v[256];        // their partial sums, when they number at most 256
    int dead[64];
    int flag;
};

// The previous iteration's closing, spread over the tiles of a launch: tile
// x of column block y closes restarts 64 y + x, 64 y + x + tiles, ... (one
// each when there are 64 row tiles).  Its threads load the restarts' partial
// sums of every row tile at the start, beside the tile's own operands; one
// thread per (restart, quantity) adds them in tile order 0 .. tiles - 1 --
// the order of lowp_close, so the sums are the same bit for bit -- and the
// restarts are finished in the epilogue.
struct FusedClose {
    const double* partials;     // nullptr: nothing to close
    int64_t kk;
    double beta, eps;
    double* log;
    RestartState* state;
};

// The tile's slabs of J and of the restart copy, and the thread's chunk of
// a stage: row 16 u + tid / 16, bytes 16 (tid % 16), so 16 consecutive
// lanes read a row's stage as two whole cache lines.
struct FusedSlab {
    __amdgpu_buffer_rsrc_t rJ, rU;
    uint32_t voff, rowb;
    int soff, nst;
};

template <int DEPTH>
__device__ __forceinline__ void fused_fetch_j(i32x4 (&r)[8], const FusedSlab& sl, int st) {
    const uint32_t o = sl.voff + static_cast<uint32_t>(st) * kFusedStage;
#pragma unroll
    for (int u = 0; u < 4; ++u) r[u] = __builtin_amdgcn_raw_buffer_load_b128(sl.rJ, o, u * 16 * sl.rowb, 0);
}

template <int DEPTH>
__device__ __forceinline__ void fused_fetch_u(i32x4 (&r)[8], const FusedSlab& sl, int st) {
    const uint32_t o = sl.voff + static_cast<uint32_t>(st) * kFusedStage;
#pragma unroll
    for (int u = 0; u < 4; ++u) r[4 + u] = __builtin_amdgcn_raw_buffer_load_b128(sl.rU, o, u * 16 * sl.rowb, 0);
}

// One iteration of tile (row0, col0).  ring holds DEPTH stages in flight;
// with j_ready the J halves of the first DEPTH stages are already in it
// (the resident kernel requests them before its barrier: J does not change).
// Its partial sums go to row tile `tx` of `partials`.
// RS_PRE: the FP8 row scales are requested with the other epilogue inputs
// at the start (registers permitting), else read in the epilogue.  CLOSE:
// the tile also closes restarts of the previous iteration (fc).
template <int PREC, int DEPTH, bool RS_PRE, bool CLOSE>
__device__ __forceinline__ void fused_tile(FusedLds& L, i32x4 (&ring)[DEPTH][8], bool j_ready, const FusedSlab& sl,
                                           int Rp, int row0, int col0, int tx, const float* __restrict__ rscale,
                                           const float* __restrict__ U_old, float* __restrict__ U_new,
                                           typename Prec<PREC>::T* __restrict__ Ub_new,
                                           const float* __restrict__ cs_old, float* __restrict__ cs_new,
                                           double rho_q, double alpha, int R, double* __restrict__ partials,
                                           const RestartState* __restrict__ state, const FusedClose& fc) {
    using T = typename Prec<PREC>::T;
    using M = Mfma<PREC>;
    constexpr int SROW = kFusedSrow;
    constexpr int FB = M::kBytes / 2;           // fragment bytes per lane
    const int np = static_cast<int>(sl.rowb / sizeof(T));
    const int tiles = np / 64;
    // restarts this tile closes: col0 + tx + m * tiles, m < nres; their sums
    // (nres x tiles x 4) are loaded first and parked in the second stage
    // buffer, which the k loop first writes after its first barrier
    const int nres = (CLOSE && fc.partials) ? (tx < 64 ? (64 - tx + tiles - 1) / tiles : 0) : 0;
    const int ncl = nres * tiles * 4;
    // up to 256 sums (64 row tiles or fewer): one per thread, held in a
    // register through the k loop and added in the epilogue, so their
    // latency is off the path; more (np > 4096) are parked and added before
    // the k loop, in the second stage buffer, which the loop first writes
    // after its first barrier
    const bool cl_small = ncl <= MT;
    double clv = 0.0;
    if (cl_small && static_cast<int>(threadIdx.x) < ncl) {
        const int idx = threadIdx.x;
        const int m = idx / (tiles * 4), t = (idx >> 2) % tiles, q = idx & 3;
        clv = fc.partials[(static_cast<size_t>(t) * Rp + col0 + tx + m * tiles) * 4 + q];
    }
    float* const sred = reinterpret_cast<float*>(L.stage);
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = tid >> 6;
    const int wr = wave >> 1, wc = wave & 1;
    const int mycol = col0 + (tid & 63);
    // The inputs of the epilogue and of the liveness test are requested
    // first, the first DEPTH stages right after them, so the latency of all
    // of it overlaps: lane column j, rows 8*(v/4) + 4*(lane/32) + v%4 of
    // sub-tile row wr.
    const int jl = wc * 32 + (lane & 31);
    const int j = col0 + jl;
    const int done_m = (tid < 64 && mycol < R) ? state[mycol].done : 1;
    const int done_j = j < R ? state[j].done : 1;
    if (!j_ready) {
#pragma unroll
        for (int p = 0; p < DEPTH; ++p) fused_fetch_j<DEPTH>(ring[p], sl, p);
    }
    // every row holds at least DEPTH stages (lowp_shape_valid)
#pragma unroll
    for (int p = 0; p < DEPTH; ++p) fused_fetch_u<DEPTH>(ring[p], sl, p);
    float uo_pre[16];
#pragma unroll
    for (int v = 0; v < 16; ++v) {
        const int il = wr * 32 + 8 * (v >> 2) + 4 * (lane >> 5) + (v & 3);
        uo_pre[v] = U_old[static_cast<size_t>(row0 + il) * Rp + j];
    }
    float c_in = 1.0f;
    float rs_pre[16];
    if constexpr (PREC == 1) {
        c_in = cs_old[j];
        if constexpr (RS_PRE) {
#pragma unroll
            for (int v = 0; v < 16; ++v)
                rs_pre[v] = rscale[row0 + wr * 32 + 8 * (v >> 2) + 4 * (lane >> 5) + (v & 3)];
        }
    }
    if (tid < 64) L.dead[tid] = done_m;
    if (!cl_small) {
        double* const cl = reinterpret_cast<double*>(L.stage + 2 * 64 * SROW);
        for (int idx = tid; idx < ncl; idx += MT) {
            const int m = idx / (tiles * 4), t = (idx >> 2) % tiles, q = idx & 3;
            cl[idx] = fc.partials[(static_cast<size_t>(t) * Rp + col0 + tx + m * tiles) * 4 + q];
        }
    }
    const bool block_live = __syncthreads_or(!done_m) != 0;
    if (!cl_small && tid < nres * 4) {
        const double* const cl = reinterpret_cast<const double*>(L.stage + 2 * 64 * SROW);
        const int m = tid >> 2, q = tid & 3;
        double sum = 0.0;
        for (int t = 0; t < tiles; ++t) sum = dadd(sum, cl[(m * tiles + t) * 4 + q]);
        L.close_s[m][q] = sum;
    }

    f32x16 acc[2][2];
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b) acc[a][b] = f32x16{};
    if (block_live) {
        const int fo = (lane & 31) * SROW + (lane >> 5) * FB;
        // registers of stage st to LDS buffer st % 2, then the refetch DEPTH
        // stages ahead into the same registers
        auto put = [&](i32x4 (&r)[8], int st, bool refetch) {
            char* A = L.stage + (st & 1) * 2 * 64 * SROW;
            char* B = A + 64 * SROW;
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                *reinterpret_cast<i32x4*>(A + sl.soff + u * 16 * SROW) = r[u];
                *reinterpret_cast<i32x4*>(B + sl.soff + u * 16 * SROW) = r[4 + u];
            }
            if (refetch) {
                fused_fetch_j<DEPTH>(r, sl, st + DEPTH);
                fused_fetch_u<DEPTH>(r, sl, st + DEPTH);
            }
        };
        // this wavefront's MFMA steps of stage st (wave, wave + 4, ...)
        auto compute = [&](int st) {
            const char* A = L.stage + (st & 1) * 2 * 64 * SROW;
            const char* B = A + 64 * SROW;
#pragma unroll
            for (int ks = wave; ks < kFusedStage / M::kBytes; ks += 4) {
                const int kb = ks * M::kBytes;
                const auto a0 = M::load(A + fo + kb);
                const auto a1 = M::load(A + 32 * SROW + fo + kb);
                const auto b0 = M::load(B + fo + kb);
                const auto b1 = M::load(B + 32 * SROW + fo + kb);
                acc[0][0] = M::step(a0, b0, acc[0][0]);
                acc[0][1] = M::step(a0, b1, acc[0][1]);
                acc[1][0] = M::step(a1, b0, acc[1][0]);
                acc[1][1] = M::step(a1, b1, acc[1][1]);
            }
        };
        // stage st + 1 goes to LDS while stage st is multiplied (the other
        // buffer, free since the barrier that ended stage st - 1), one
        // barrier per stage
        const int nst = sl.nst;
        put(ring[0], 0, DEPTH < nst);
        __syncthreads();
        int s0 = 0;
        for (; s0 + 2 * DEPTH < nst; s0 += DEPTH) {
#pragma unroll
            for (int p = 0; p < DEPTH; ++p) {
                put(ring[(p + 1) % DEPTH], s0 + p + 1, true);
                compute(s0 + p);
                __syncthreads();
            }
        }
#pragma unroll
        for (int q = 0; q < 2 * DEPTH; ++q) {
            const int st = s0 + q;
            if (st < nst) {
                if (st + 1 < nst) put(ring[(q + 1) % DEPTH], st + 1, st + 1 + DEPTH < nst);
                compute(st);
                __syncthreads();
            }
        }
    }
    __syncthreads();                            // the stage buffers are reused below
    // ---- reduction of the four partial tiles: wavefront w keeps sub-tile
    // (wr, wc) = (w / 2, w % 2), summed over wavefronts 0..3 in order
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b)
#pragma unroll
            for (int v = 0; v < 16; ++v) sred[((wave * 4 + a * 2 + b) * 16 + v) * 64 + lane] = acc[a][b][v];
    __syncthreads();
    f32x16 tile;
#pragma unroll
    for (int v = 0; v < 16; ++v) {
        float t = sred[((0 * 4 + wave) * 16 + v) * 64 + lane];
#pragma unroll
        for (int w = 1; w < 4; ++w) t += sred[((w * 4 + wave) * 16 + v) * 64 + lane];
        tile[v] = t;
    }
    __syncthreads();                            // sred is reused below
    if (cl_small && tid < ncl) L.close_v[tid] = clv;

    // ---- epilogue: lane holds column j, rows 8*(v/4) + 4*(lane/32) + v%4
    const bool live = j < R && !done_j;
    double part[4] = {0.0, 0.0, 0.0, 0.0};      // u^4, u^2, u z, (du)^2
    // FP8: scale of the copy read by this product and of the one written now
    float c_out = 1.0f, inv_c = 1.0f;
    if constexpr (PREC == 1) {
        c_out = live ? next_colscale(c_in, rho_q, alpha) : c_in;
        // the copy is u times a reciprocal of its scale (v_rcp_f32, within an
        // ulp): the next product multiplies by the scale itself, and the
        // carried bound has a margin far beyond an ulp
        inv_c = __builtin_amdgcn_rcpf(c_out);
        if (row0 == 0 && wr == 0 && lane < 32) cs_new[j] = c_out;
    }
    // transposed low-precision tile: row jl holds rows row0 .. row0+63 of restart j
    T* tileT = reinterpret_cast<T*>(L.stage);
    constexpr int TROW = 64 + 16 / static_cast<int>(sizeof(T));   // padded row, in elements
#pragma unroll
    for (int v = 0; v < 16; ++v) {
        const int il = wr * 32 + 8 * (v >> 2) + 4 * (lane >> 5) + (v & 3);
        const int i = row0 + il;
        const size_t ij = static_cast<size_t>(i) * Rp + j;
        const double uo = static_cast<double>(uo_pre[v]);
        double z = static_cast<double>(tile[v]);
        if (PREC == 1)
            z = dmul(dmul(z, static_cast<double>(RS_PRE ? rs_pre[v] : rscale[i])), static_cast<double>(c_in));
        float un = uo_pre[v];
        if (live) {
            // the argument in FP64, its cube root in FP32: the result is
            // stored in FP32 either way
            un = cbrtf(static_cast<float>(dadd(z, dmul(alpha, uo))));
            const double d = dsub(static_cast<double>(un), uo);
            const double u2 = dmul(uo, uo);
            part[0] = dadd(part[0], dmul(u2, u2));
            part[1] = dadd(part[1], u2);
            part[2] = dadd(part[2], dmul(uo, z));
            part[3] = dadd(part[3], dmul(d, d));
            // a stopped restart is never written again: its last iterate
            // stays in the buffer the next iteration would otherwise overwrite
            U_new[ij] = un;
        }
        tileT[jl * TROW + il] = to_lowp<PREC>(PREC == 1 ? un * inv_c : un);
    }
    // rows of a column: lanes l and l + 32, then the two row halves of the tile
#pragma unroll
    for (int q = 0; q < 4; ++q) part[q] = dadd(part[q], __shfl_xor(part[q], 32, 64));
    if (lane < 32) {
#pragma unroll
        for (int q = 0; q < 4; ++q) L.red[wr][jl][q] = part[q];
    }
    __syncthreads();
    if (cl_small && (tid & 63) < nres) {
        // quantity q = wave, restart m = lane: four chains per restart at once,
        // each in tile order
        const int m = tid & 63, q = tid >> 6;
        double sum = 0.0;
        for (int t = 0; t < tiles; ++t) sum = dadd(sum, L.close_v[(m * tiles + t) * 4 + q]);
        L.close_s[m][q] = sum;
    }
    {
        // 64 restart rows of 64 * sizeof(T) bytes, in 16-byte chunks
        constexpr int CPR = 64 * static_cast<int>(sizeof(T)) / 16;
        for (int c = tid; c < 64 * CPR; c += MT) {
            const int r = c / CPR, ch = c % CPR;
            if (L.dead[r]) continue;
            const i32x4 v = *reinterpret_cast<const i32x4*>(reinterpret_cast<const char*>(tileT + r * TROW) + ch * 16);
            *reinterpret_cast<i32x4*>(reinterpret_cast<char*>(Ub_new + static_cast<size_t>(col0 + r) * np + row0) +
                                      ch * 16) = v;
        }
    }
    // partial sums of this row tile, closed after the iteration
    if (tid < 64) {
        double* p = partials + (static_cast<size_t>(tx) * Rp + col0 + tid) * 4;
#pragma unroll
        for (int q = 0; q < 4; ++q) p[q] = dadd(L.red[0][tid][q], L.red[1][tid][q]);
    }
    __syncthreads();                            // LDS is reused by the next iteration
    if (tid < nres) {
        // the restart's stop flag as this launch read it (only this tile
        // writes its state here)
        const int off = tx + tid * tiles;
        const double S[4] = {L.close_s[tid][0], L.close_s[tid][1], L.close_s[tid][2], L.close_s[tid][3]};
        lowp_close_restart(S, col0 + off, R, fc.kk, alpha, fc.beta, fc.eps, fc.log, fc.state, L.dead[off]);
    }
}

template <int PREC>
__device__ __forceinline__ FusedSlab fused_slab(int np, int row0, int col0, const typename Prec<PREC>::T* Jq,
                                                const typename Prec<PREC>::T* Ub_old) {
    using T = typename Prec<PREC>::T;
    FusedSlab sl;
    sl.rowb = static_cast<uint32_t>(np) * sizeof(T);
    sl.rJ = slab_rsrc(reinterpret_cast<const char*>(Jq) + static_cast<size_t>(row0) * sl.rowb, 64 * sl.rowb);
    sl.rU = slab_rsrc(reinterpret_cast<const char*>(Ub_old) + static_cast<size_t>(col0) * sl.rowb, 64 * sl.rowb);
    sl.voff = (threadIdx.x >> 4) * sl.rowb + (threadIdx.x & 15) * 16;
    sl.soff = (threadIdx.x >> 4) * kFusedSrow + (threadIdx.x & 15) * 16;
    sl.nst = static_cast<int>(sl.rowb / kFusedStage);
    return sl;
}

// One launch per iteration; its tiles also close the previous iteration
// (FusedClose).  A tile may read a restart's state while another tile of the
// launch stops it; the restart is then updated once more into the buffer
// after its last iterate, which stays where iters_done says.
template <int PREC, int DEPTH>
__global__ __launch_bounds__(MT) __attribute__((amdgpu_waves_per_eu(2))) void lowp_fused_kernel(
    int np, int Rp, const typename Prec<PREC>::T* __restrict__ Jq, const float* __restrict__ rscale,
    const float* __restrict__ U_old, float* __restrict__ U_new,
    const typename Prec<PREC>::T* __restrict__ Ub_old, typename Prec<PREC>::T* __restrict__ Ub_new,
    const float* __restrict__ cs_old, float* __restrict__ cs_new, double rho_q,
    double alpha, double beta, double eps, int R, int64_t k, const double* __restrict__ partials_prev,
    double* __restrict__ partials, double* __restrict__ log, RestartState* __restrict__ state) {
    __shared__ FusedLds L;
    const int row0 = blockIdx.x * 64, col0 = blockIdx.y * 64;
    const FusedSlab sl = fused_slab<PREC>(np, row0, col0, Jq, Ub_old);
    const FusedClose fc{k > 0 ? partials_prev : nullptr, k - 1, beta, eps, log, state};
    i32x4 ring[DEPTH][8];
    fused_tile<PREC, DEPTH, true, true>(L, ring, false, sl, Rp, row0, col0, blockIdx.x, rscale, U_old, U_new, Ub_new, cs_old,
                            cs_new, rho_q, alpha, R, partials, state, fc);
}

// ---- the fused iteration resident for the whole run ---------------------
//
// One cooperative launch: workgroup t owns a tile for every iteration (the
// column blocks of a row tile on one XCD, so the J slab they share meets in
// one L2), and closes restarts of the previous iteration as the launches'
// tiles do.  Between iterations a grid barrier: every wave drains its
// stores, then one thread per workgroup releases at device scope (the
// restart copy crosses XCDs, whose L2 caches are not coherent with each
// other), counts the workgroup in (a counter per group of workgroups, then
// one for the groups) and polls its group's release word, and acquires at
// device scope.  The J halves of the next iteration's first stages are
// requested before the barrier: J does not change.  A restart stopped by
// the closing in iteration k is seen from iteration k + 1 on, as with the
// launches, so both give the same iterates bit for bit.  Every wait is
// bounded: a workgroup that polls too long marks every restart aborted and
// publishes a stop that every other one sees at its next poll.
struct LowpResArgs {
    int np, Rp, R, tiles, cblocks;
    int64_t iters;
    const void* Jq;
    const float* rscale;
    float* U[3];
    void* Ub[3];
    float* cs[3];
    double rho_q, alpha, beta, eps;
    double* partials[2];
    double* log;
    RestartState* state;
    ResidentSync* sync;
};

constexpr unsigned int kLowpSpinLimit = 1u << 22;

__device__ bool lowp_barrier(ResidentSync* sy, unsigned int gen, RestartState* st, int R, int* flag) {
    asm volatile("s_waitcnt vmcnt(0) lgkmcnt(0)" ::: "memory");
    __syncthreads();
    if (threadIdx.x == 0) {
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
        const unsigned int G = gridDim.x;
        const unsigned int g = blockIdx.x & 7u;
        const unsigned int per = (G - g + 7u) / 8u;
        const unsigned int groups = G < 8u ? G : 8u;
        auto add = [](unsigned int* p) {
            return __hip_atomic_fetch_add(p, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        };
        auto put = [](unsigned int* p, unsigned int v) {
            __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        };
        if (add(&sy->grp[g * kTicketStride]) == gen * per - 1u) {
            if (add(&sy->top[0]) == gen * groups - 1u)
                for (unsigned int q = 0; q < groups; ++q) put(&sy->flag[q * kTicketStride], gen);
        }
        unsigned long long* f = reinterpret_cast<unsigned long long*>(sy->flag + g * kTicketStride);
        unsigned int spins = 0;
        int ok = 1;
        for (;;) {
            const unsigned long long v = __hip_atomic_load(f, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            if (static_cast<unsigned int>(v >> 32) != 0u) { ok = 0; break; }
            if (static_cast<unsigned int>(v) >= gen) break;
            if (++spins > kLowpSpinLimit) {
                for (int r = 0; r < R; ++r) {
                    __hip_atomic_store(&st[r].aborted, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                    __hip_atomic_store(&st[r].done, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                }
                for (unsigned int q = 0; q < groups; ++q) put(&sy->flag[q * kTicketStride + 1], 2u);
                ok = 0;
                break;
            }
            __builtin_amdgcn_s_sleep(1);
        }
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
        *flag = ok;
    }
    __syncthreads();
    return *flag != 0;
}

template <int PREC, int DEPTH>
__global__ __launch_bounds__(MT) void lowp_resident_kernel(LowpResArgs a) {
    using T = typename Prec<PREC>::T;
    __shared__ FusedLds L;
    const int b = blockIdx.x;
    // tile: the cblocks column blocks of a row tile on one XCD (workgroup b
    // runs on XCD b mod 8 under round-robin dispatch)
    int tx, ty;
    if ((a.tiles & 7) == 0) {
        const int x8 = b >> 3;
        tx = (b & 7) + 8 * (x8 / a.cblocks);
        ty = x8 % a.cblocks;
    } else {
        tx = b % a.tiles;
        ty = b / a.tiles;
    }
    const int row0 = tx * 64, col0 = ty * 64;
    const T* Jq = static_cast<const T*>(a.Jq);
    i32x4 ring[DEPTH][8];
    for (int64_t k = 0; k < a.iters; ++k) {
        const int o = static_cast<int>(k % 3), n = static_cast<int>((k + 1) % 3);
        if (k > 0 && !lowp_barrier(a.sync, static_cast<unsigned int>(k), a.state, a.R, &L.flag)) return;
        const FusedSlab sl = fused_slab<PREC>(a.np, row0, col0, Jq, static_cast<const T*>(a.Ub[o]));
        const FusedClose fc{k > 0 ? a.partials[(k - 1) & 1] : nullptr, k - 1, a.beta, a.eps, a.log, a.state};
        fused_tile<PREC, DEPTH, true, true>(L, ring, k > 0, sl, a.Rp, row0, col0, tx, a.rscale, a.U[o], a.U[n],
                                            static_cast<T*>(a.Ub[n]), a.cs[o], a.cs[n], a.rho_q, a.alpha, a.R,
                                            a.partials[k & 1], a.state, fc);
        if (k + 1 < a.iters) {
#pragma unroll
            for (int p = 0; p < DEPTH; ++p) fused_fetch_j<DEPTH>(ring[p], sl, p);
        }
    }
}

// ---- J held in LDS: the product split over k across the device ----------
//
// One cooperative launch for the whole run, one workgroup of eight
// wavefronts per compute unit.  Workgroup (rb, kb) holds rows 128 rb ..
// 128 rb + 127 of J, k bytes [KSB kb, KSB (kb + 1)), in LDS from its start
// to its end (128 KB at KSB = 1024), so an iteration streams only the
// low-precision restart copy (L2-resident: 2 MB at n = 4096, 256 restarts)
// instead of a J slab per output tile.  An iteration:
//   product   every wavefront owns 32-restart blocks (wave, wave + 8, ...)
//             and, per block, the 128 x 32 FP32 partial product over the
//             slice: 4 MFMA chains of 32 rows, A from LDS, B straight from
//             memory (each copy row read by one wavefront only), written to
//             P[kb] (np x Rp, FP32);
//   closing   of the previous iteration: restarts b, b + G, ... of
//             workgroup b, the row tiles' sums added in tile order as
//             lowp_close does;
//   barrier
//   update    the 64 x 64 tiles of rows 128 rb .. 128 rb + 127, split over
//             the workgroups of row block rb: the KB partial products added
//             in slice order, the update, the FP32 master and the
//             low-precision copy, the row tile's FP64 partial sums;
//   barrier   (before the next product reads the new copy).
// A row block's workgroups sit on one XCD when the row blocks split evenly
// over the eight XCDs (workgroup b on XCD b mod 8), so the partial products
// an update tile adds were written through its own L2.
//
// k order inside the product: the slice's rows are read in 128-byte groups;
// lane half h of a group holds bytes 64 h .. 64 h + 63 of its row, in 16-byte
// (BF16) or 32-byte (FP8) pieces, one per MFMA step, and reads A the same
// way, so k pairs with k.  Every lane loads its 64 bytes of a group as four
// 16-byte pieces of one row segment, D groups ahead.
constexpr int HT = 512;                        // threads per workgroup
constexpr int kHeldRows = 128;

template <int NG>
struct HeldLds {
    static constexpr int kPitch = NG * 128 + 16;
    __attribute__((aligned(16))) char J[kHeldRows * kPitch];
    // update: [8][64][4] doubles of partial sums, then the transposed copy;
    // closing: 512 staged sums and the closed restarts' totals
    __attribute__((aligned(16))) char scratch[16384];
    int dead[64];
    int flag;
};

struct LowpHeldArgs {
    int np, Rp, R, rblocks, kslices;
    int64_t iters;
    const void* Jq;
    const float* rscale;
    float* U[3];
    void* Ub[3];
    float* cs[3];
    double rho_q, alpha, beta, eps;
    float* P;
    double* partials[2];
    double* log;
    RestartState* state;
    ResidentSync* sync;
};

// One 64 x 64 update tile (row tile rt, column block cb) with 512 threads:
// lane l of wavefront w holds restart 64 cb + l and rows 64 rt + 8 w ..
// 64 rt + 8 w + 7.  The S partial products are added in slice order, then
// as lowp_update_kernel.
template <int PREC>
__device__ __forceinline__ void held_update_tile(char* scratch, int* sdead, int np, int Rp, int S, int rt, int cb,
                                                 const float* __restrict__ P, const float* __restrict__ rscale,
                                                 const float* __restrict__ U_old, float* __restrict__ U_new,
                                                 typename Prec<PREC>::T* __restrict__ Ub_new,
                                                 const float* __restrict__ cs_old, float* __restrict__ cs_new,
                                                 double rho_q, double alpha, int R, double* __restrict__ partials,
                                                 const RestartState* __restrict__ state) {
    using T = typename Prec<PREC>::T;
    constexpr int TROW = 64 + 16 / static_cast<int>(sizeof(T));
    const int tid = threadIdx.x;
    const int jl = tid & 63, rg = tid >> 6;
    const int row0 = rt * 64, col0 = cb * 64;
    const int j = col0 + jl;
    const int i0 = row0 + rg * 8;
    const size_t base = static_cast<size_t>(i0) * Rp + j;
    const size_t pstride = static_cast<size_t>(np) * Rp;
    float uo[8], zs[8][8];
#pragma unroll
    for (int v = 0; v < 8; ++v) uo[v] = U_old[base + static_cast<size_t>(v) * Rp];
#pragma unroll
    for (int sp = 0; sp < 8; ++sp)
        if (sp < S) {
#pragma unroll
            for (int v = 0; v < 8; ++v) zs[sp][v] = P[sp * pstride + base + static_cast<size_t>(v) * Rp];
        }
    const int dead = j < R ? state[j].done : 1;
    if (tid < 64) sdead[tid] = dead;
    const bool live = !dead;
    float c_in = 1.0f, c_out = 1.0f, inv_c = 1.0f;
    if constexpr (PREC == 1) {
        c_in = cs_old[j];
        c_out = live ? next_colscale(c_in, rho_q, alpha) : c_in;
        // the copy is u times a reciprocal of its scale (v_rcp_f32, within an
        // ulp); the carried bound has a margin far beyond an ulp
        inv_c = __builtin_amdgcn_rcpf(c_out);
        if (row0 == 0 && rg == 0) cs_new[j] = c_out;
    }
    double part[4] = {0.0, 0.0, 0.0, 0.0};      // u^4, u^2, u z, (du)^2
    T low[8];
#pragma unroll
    for (int v = 0; v < 8; ++v) {
        const int i = i0 + v;
        float z32 = zs[0][v];
#pragma unroll
        for (int sp = 1; sp < 8; ++sp)
            if (sp < S) z32 += zs[sp][v];
        const double u = static_cast<double>(uo[v]);
        double z = static_cast<double>(z32);
        if (PREC == 1) z = dmul(dmul(z, static_cast<double>(rscale[i])), static_cast<double>(c_in));
        float un = uo[v];
        if (live) {
            // the argument in FP64, its cube root in FP32
            un = cbrtf(static_cast<float>(dadd(z, dmul(alpha, u))));
            const double d = dsub(static_cast<double>(un), u);
            const double u2 = dmul(u, u);
            part[0] = dadd(part[0], dmul(u2, u2));
            part[1] = dadd(part[1], u2);
            part[2] = dadd(part[2], dmul(u, z));
            part[3] = dadd(part[3], dmul(d, d));
            U_new[base + static_cast<size_t>(v) * Rp] = un;
        }
        low[v] = to_lowp<PREC>(PREC == 1 ? un * inv_c : un);
    }
    double (*red)[64][4] = reinterpret_cast<double (*)[64][4]>(scratch);
#pragma unroll
    for (int q = 0; q < 4; ++q) red[rg][jl][q] = part[q];
    __syncthreads();
    // the row tile's partial sums (row groups in order)
    if (tid < 64) {
        double* p = partials + (static_cast<size_t>(rt) * Rp + col0 + tid) * 4;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            double sum = red[0][tid][q];
#pragma unroll
            for (int g = 1; g < 8; ++g) sum = dadd(sum, red[g][tid][q]);
            p[q] = sum;
        }
    }
    __syncthreads();
    T* tileT = reinterpret_cast<T*>(scratch);
#pragma unroll
    for (int v = 0; v < 8; ++v) tileT[jl * TROW + rg * 8 + v] = low[v];
    __syncthreads();
    {
        // 64 restart rows of 64 * sizeof(T) bytes, in 16-byte chunks
        constexpr int CPR = 64 * static_cast<int>(sizeof(T)) / 16;
        for (int c = tid; c < 64 * CPR; c += HT) {
            const int r = c / CPR, ch = c % CPR;
            if (sdead[r]) continue;
            const i32x4 val = *reinterpret_cast<const i32x4*>(reinterpret_cast<const char*>(tileT + r * TROW) + ch * 16);
            *reinterpret_cast<i32x4*>(reinterpret_cast<char*>(Ub_new + static_cast<size_t>(col0 + r) * np + row0) +
                                      ch * 16) = val;
        }
    }
    __syncthreads();                            // scratch and sdead are reused
}

template <int PREC, int NG>
__global__ __launch_bounds__(HT) void lowp_held_kernel(LowpHeldArgs a) {
    using T = typename Prec<PREC>::T;
    using M = Mfma<PREC>;
    constexpr int KSB = NG * 128;               // k bytes per row held
    constexpr int PITCH = HeldLds<NG>::kPitch;
    constexpr int D = NG < 4 ? NG : 4;          // groups in flight per lane
    constexpr int FB = M::kBytes / 2;           // fragment bytes per lane
    constexpr int KPG = 64 / FB;                // MFMA steps per 128-byte group
    __shared__ HeldLds<NG> L;
    const int b = blockIdx.x, G = gridDim.x;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int np = a.np, Rp = a.Rp, KB = a.kslices;
    int rb, kb;
    if (a.rblocks % 8 == 0 && G % 8 == 0) {
        const int x = b & 7, m = b >> 3;
        rb = x * (a.rblocks / 8) + m / KB;
        kb = m % KB;
    } else {
        rb = b / KB;
        kb = b % KB;
    }
    const uint32_t rowb = static_cast<uint32_t>(np) * sizeof(T);
    {
        const char* src = static_cast<const char*>(a.Jq) + static_cast<size_t>(rb) * kHeldRows * rowb +
                          static_cast<size_t>(kb) * KSB;
        for (int c = tid; c < kHeldRows * (KSB / 16); c += HT) {
            const int r = c / (KSB / 16), ch = c % (KSB / 16);
            *reinterpret_cast<i32x4*>(L.J + r * PITCH + ch * 16) =
                *reinterpret_cast<const i32x4*>(src + static_cast<size_t>(r) * rowb + ch * 16);
        }
    }
    __syncthreads();
    // restarts this workgroup closes: b + G m, m < nres
    const int nres = b < Rp ? (Rp - b + G - 1) / G : 0;
    const int tiles = np / 64;
    const int ncl = nres * tiles * 4;
    const int CB = Rp / 64;
    const int fo = (lane & 31) * PITCH + (lane >> 5) * 64;
    for (int64_t k = 0; k < a.iters; ++k) {
        const int o = static_cast<int>(k % 3), n = static_cast<int>((k + 1) % 3);
        const double* pprev = a.partials[(k + 1) & 1];
        // the first 512 sums this workgroup closes, requested now and added
        // after the product (value (t nres + m) 4 + q: row tile t, restart
        // b + G m, quantity q)
        double clv = 0.0;
        if (k > 0 && tid < ncl) {
            const int t = tid / (nres * 4), m = (tid >> 2) % nres, q = tid & 3;
            clv = pprev[(static_cast<size_t>(t) * Rp + b + G * m) * 4 + q];
        }
        // ---- product
        const __amdgpu_buffer_rsrc_t rU = slab_rsrc(a.Ub[o], static_cast<uint32_t>(Rp) * rowb);
        const __amdgpu_buffer_rsrc_t rP =
            slab_rsrc(a.P + static_cast<size_t>(kb) * np * Rp, static_cast<uint32_t>(np) * static_cast<uint32_t>(Rp) * 4u);
        for (int blk = wave; blk < Rp / 32; blk += 8) {
            const uint32_t voff = static_cast<uint32_t>(blk * 32 + (lane & 31)) * rowb +
                                  static_cast<uint32_t>(kb * KSB + (lane >> 5) * 64);
            i32x4 ring[D][4];
#pragma unroll
            for (int p = 0; p < D; ++p)
#pragma unroll
                for (int c = 0; c < 4; ++c)
                    ring[p][c] = __builtin_amdgcn_raw_buffer_load_b128(rU, voff + p * 128 + c * 16, 0, 0);
            f32x16 acc[4];
#pragma unroll
            for (int r = 0; r < 4; ++r) acc[r] = f32x16{};
            // D groups per trip, the ring slot of each known at compile time;
            // the A fragments of the next MFMA step are read while this
            // step's four MFMAs run, and the scheduler is kept from hoisting
            // further reads (which would only take registers)
            typename M::frag af[2][4];
            auto read_a = [&](typename M::frag (&d)[4], int g, int c) {
#pragma unroll
                for (int r = 0; r < 4; ++r) d[r] = M::load(L.J + r * 32 * PITCH + fo + g * 128 + c * FB);
            };
            read_a(af[0], 0, 0);
#pragma unroll 1
            for (int g0 = 0; g0 < NG; g0 += D) {
                const bool refetch = g0 + D < NG;
#pragma unroll
                for (int p = 0; p < D; ++p) {
                    const int g = g0 + p;
                    i32x4 (&bq)[4] = ring[p];
#pragma unroll
                    for (int c = 0; c < KPG; ++c) {
                        const int cur = (p * KPG + c) & 1;
                        // the next step: (g, c + 1) or (g + 1, 0); past the
                        // slice end it rereads the first step, unused
                        const int gn = c + 1 < KPG ? g : g + 1;
                        const int cn = c + 1 < KPG ? c + 1 : 0;
                        read_a(af[cur ^ 1], gn < NG ? gn : 0, cn);
                        typename M::frag bf;
                        if constexpr (PREC == 0) bf = __builtin_bit_cast(bf16x8, bq[c]);
                        else bf = __builtin_shufflevector(bq[2 * c], bq[2 * c + 1], 0, 1, 2, 3, 4, 5, 6, 7);
#pragma unroll
                        for (int r = 0; r < 4; ++r) acc[r] = M::step(af[cur][r], bf, acc[r]);
                        __builtin_amdgcn_sched_barrier(0);
                    }
                    if (refetch) {
#pragma unroll
                        for (int c = 0; c < 4; ++c)
                            bq[c] = __builtin_amdgcn_raw_buffer_load_b128(rU, voff + (g + D) * 128 + c * 16, 0, 0);
                    }
                }
            }
            // C layout: lane column l % 32, rows 8 (v / 4) + 4 (l / 32) + v % 4;
            // the row step in the scalar offset, so no store needs an
            // address register of its own
            const uint32_t Rp4 = static_cast<uint32_t>(Rp) * 4u;
            const uint32_t vo = static_cast<uint32_t>(rb * kHeldRows + 4 * (lane >> 5)) * Rp4 +
                                static_cast<uint32_t>(blk * 32 + (lane & 31)) * 4u;
#pragma unroll
            for (int r = 0; r < 4; ++r)
#pragma unroll
                for (int v = 0; v < 16; ++v) {
                    // the element is read into a scalar first: a bit cast of
                    // the vector element itself was compiled as element 0
                    const float e = acc[r][v];
                    __builtin_amdgcn_raw_buffer_store_b32(__float_as_uint(e), rP,
                                                          vo + static_cast<uint32_t>(r * 32) * Rp4,
                                                          static_cast<uint32_t>(8 * (v >> 2) + (v & 3)) * Rp4, 0);
                }
        }
        // ---- closing of iteration k - 1 (the order of lowp_close)
        if (k > 0 && nres > 0) {
            double* cv = reinterpret_cast<double*>(L.scratch);
            double* tot = cv + HT;
            const int m = tid >> 2, q = tid & 3;
            const bool summer = tid < nres * 4;
            double run = 0.0;
            for (int base = 0; base < ncl; base += HT) {
                double v = clv;
                if (base > 0) {
                    v = 0.0;
                    const int idx = base + tid;
                    if (idx < ncl) {
                        const int t = idx / (nres * 4), mm = (idx >> 2) % nres, qq = idx & 3;
                        v = pprev[(static_cast<size_t>(t) * Rp + b + G * mm) * 4 + qq];
                    }
                }
                __syncthreads();
                cv[tid] = v;
                __syncthreads();
                if (summer && ncl <= HT) {
#pragma unroll 16
                    for (int t = 0; t < tiles; ++t) run = dadd(run, cv[(t * nres + m) * 4 + q]);
                } else if (summer) {
                    const int t0 = base / (nres * 4);
                    const int t1 = (base + HT + nres * 4 - 1) / (nres * 4);
                    for (int t = t0; t < t1 && t < tiles; ++t) {
                        const int idx = (t * nres + m) * 4 + q;
                        if (idx >= base && idx < base + HT) run = dadd(run, cv[idx - base]);
                    }
                }
            }
            if (summer) tot[tid] = run;
            __syncthreads();
            if (tid < nres) {
                const double S[4] = {tot[tid * 4], tot[tid * 4 + 1], tot[tid * 4 + 2], tot[tid * 4 + 3]};
                lowp_close_restart(S, b + G * tid, a.R, k - 1, a.alpha, a.beta, a.eps, a.log, a.state);
            }
        }
        if (!lowp_barrier(a.sync, static_cast<unsigned int>(2 * k + 1), a.state, a.R, &L.flag)) return;
        // ---- update: tiles 2 rb + l % 2 (row) x l / 2 (column block), l = kb, kb + KB, ...
        for (int l = kb; l < 2 * CB; l += KB)
            held_update_tile<PREC>(L.scratch, L.dead, np, Rp, KB, 2 * rb + (l & 1), l >> 1, a.P, a.rscale, a.U[o],
                                   a.U[n], static_cast<T*>(a.Ub[n]), a.cs[o], a.cs[n], a.rho_q, a.alpha, a.R,
                                   a.partials[k & 1], a.state);
        if (k + 1 < a.iters && !lowp_barrier(a.sync, static_cast<unsigned int>(2 * k + 2), a.state, a.R, &L.flag))
            return;
    }
}

// ---- the update: sum of the splits, eq:FPE in u, partial sums ----------
//
// 64 rows x 64 restarts per workgroup: lane l of wavefront w holds restart
// column l and rows 16 w .. 16 w + 15, so every load and store of a row
// covers 64 consecutive restarts.  The update of each entry (its argument
// z + alpha u in FP64, the cube root in FP32, the precision it is stored
// in), the FP32 master store and the low-precision copy (transposed through
// LDS and written in whole rows), then the restart's FP64 partial sums of
// the row tile, which the next product launch closes.  Nothing waits on the
// restart states: the loads of the iterate and of the S partial tiles are
// issued with them, and a stopped restart only discards what it loaded.
template <int PREC, int S>
__global__ __launch_bounds__(MT) void lowp_update_kernel(
    int np, int Rp, const float* __restrict__ P, const float* __restrict__ rscale,
    const float* __restrict__ U_old, float* __restrict__ U_new, typename Prec<PREC>::T* __restrict__ Ub_new,
    const float* __restrict__ cs_old, float* __restrict__ cs_new, double rho_q, double alpha,
    int R, double* __restrict__ partials, const RestartState* __restrict__ state) {
    using T = typename Prec<PREC>::T;
    constexpr int TROW = 64 + 16 / static_cast<int>(sizeof(T));   // padded row of the transposed copy
    __shared__ __attribute__((aligned(16))) T tileT[64 * TROW];
    __shared__ double red[4][64][4];
    __shared__ int sdead[64];
    const int tid = threadIdx.x;
    const int jl = tid & 63, rg = tid >> 6;
    const int row0 = blockIdx.x * 64, col0 = blockIdx.y * 64;
    const int j = col0 + jl;
    const int i0 = row0 + rg * 16;
    float uo[16], zs[S][16];
    const size_t base = static_cast<size_t>(i0) * Rp + j;
#pragma unroll
    for (int v = 0; v < 16; ++v) uo[v] = U_old[base + static_cast<size_t>(v) * Rp];
#pragma unroll
    for (int sp = 0; sp < S; ++sp)
#pragma unroll
        for (int v = 0; v < 16; ++v) zs[sp][v] = P[static_cast<size_t>(sp) * np * Rp + base + static_cast<size_t>(v) * Rp];
    const int dead = j < R ? state[j].done : 1;
    if (tid < 64) sdead[tid] = dead;
    const bool live = !dead;
    // FP8: scale of the copy read by this product and of the one written now
    float c_in = 1.0f, c_out = 1.0f, inv_c = 1.0f;
    if constexpr (PREC == 1) {
        c_in = cs_old[j];
        c_out = live ? next_colscale(c_in, rho_q, alpha) : c_in;
        // the copy is u times a reciprocal of its scale (v_rcp_f32, within an
        // ulp): the next product multiplies by the scale itself, and the
        // carried bound has a margin far beyond an ulp
        inv_c = __builtin_amdgcn_rcpf(c_out);
        if (blockIdx.x == 0 && rg == 0) cs_new[j] = c_out;
    }
    double part[4] = {0.0, 0.0, 0.0, 0.0};      // u^4, u^2, u z, (du)^2
#pragma unroll
    for (int v = 0; v < 16; ++v) {
        const int i = i0 + v;
        float z32 = zs[0][v];
#pragma unroll
        for (int sp = 1; sp < S; ++sp) z32 += zs[sp][v];
        const double u = static_cast<double>(uo[v]);
        double z = static_cast<double>(z32);
        if (PREC == 1) z = dmul(dmul(z, static_cast<double>(rscale[i])), static_cast<double>(c_in));
        float un = uo[v];
        if (live) {
            // the argument in FP64, its cube root in FP32: the result is
            // stored in FP32 either way
            un = cbrtf(static_cast<float>(dadd(z, dmul(alpha, u))));
            const double d = dsub(static_cast<double>(un), u);
            const double u2 = dmul(u, u);
            part[0] = dadd(part[0], dmul(u2, u2));
            part[1] = dadd(part[1], u2);
            part[2] = dadd(part[2], dmul(u, z));
            part[3] = dadd(part[3], dmul(d, d));
            // a stopped restart is never written again: its last iterate
            // stays in the buffer the next iteration would otherwise overwrite
            U_new[base + static_cast<size_t>(v) * Rp] = un;
        }
        tileT[jl * TROW + rg * 16 + v] = to_lowp<PREC>(PREC == 1 ? un * inv_c : un);
    }
#pragma unroll
    for (int q = 0; q < 4; ++q) red[rg][jl][q] = part[q];
    __syncthreads();
    {
        // 64 restart rows of 64 * sizeof(T) bytes, in 16-byte chunks
        constexpr int CPR = 64 * static_cast<int>(sizeof(T)) / 16;
        for (int c = tid; c < 64 * CPR; c += MT) {
            const int r = c / CPR, ch = c % CPR;
            if (sdead[r]) continue;
            const i32x4 v = *reinterpret_cast<const i32x4*>(reinterpret_cast<const char*>(tileT + r * TROW) + ch * 16);
            *reinterpret_cast<i32x4*>(reinterpret_cast<char*>(Ub_new + static_cast<size_t>(col0 + r) * np + row0) +
                                      ch * 16) = v;
        }
    }
    // this row tile's partial sums (row groups in order)
    if (tid < 64) {
        double* p = partials + (static_cast<size_t>(blockIdx.x) * Rp + col0 + tid) * 4;
#pragma unroll
        for (int q = 0; q < 4; ++q)
            p[q] = dadd(dadd(dadd(red[0][tid][q], red[1][tid][q]), red[2][tid][q]), red[3][tid][q]);
    }
}

// The last iteration's closing, after the final update.
__global__ __launch_bounds__(MT) void lowp_close_kernel(const double* __restrict__ P, int tiles, int Rp, int R,
                                                        int64_t kk, double alpha, double beta, double eps,
                                                        double* __restrict__ log, RestartState* __restrict__ state) {
    __shared__ double red[64][4];
    lowp_close(P, tiles, Rp, blockIdx.x, R, kk, alpha, beta, eps, log, state, red);
}

__device__ __forceinline__ float start_u(const double* x0, int64_t i, int R, int j, double sqrt_beta) {
    return static_cast<float>(dmul(x0[i * R + j], sqrt_beta));
}

// FP8: max_i |u_ij| of the starting block, as float bits (order-preserving
// for non-negative values), combined over row chunks of 64 with atomicMax
// into colmax_bits (zeroed by the caller).
__global__ __launch_bounds__(256) void lowp_colmax_kernel(const double* __restrict__ x0, int n, int R,
                                                          double sqrt_beta,
                                                          unsigned int* __restrict__ colmax_bits) {
    const int j = blockIdx.y * 256 + threadIdx.x;
    if (j >= R) return;
    const int i0 = blockIdx.x * 64;
    const int i1 = i0 + 64 < n ? i0 + 64 : n;
    float m = 0.0f;
    for (int i = i0; i < i1; ++i) m = fmaxf(m, fabsf(start_u(x0, i, R, j, sqrt_beta)));
    atomicMax(colmax_bits + j, __float_as_uint(m));
}

// x0 (n x R, double) -> u = sqrt(beta) x in the padded FP32 master and the
// transposed low-precision copy; padding rows and restarts are zero.  FP8
// divides by the restart scale c_j = max_i |u_ij| / 448 (1 for a zero
// column) and records it.
template <int PREC>
__global__ __launch_bounds__(256) void lowp_load_kernel(const double* __restrict__ x0, int n, int R,
                                                       int np, int Rp, double sqrt_beta,
                                                       const unsigned int* __restrict__ colmax_bits,
                                                       float* __restrict__ cs, float* __restrict__ U,
                                                       typename Prec<PREC>::T* __restrict__ Ub) {
    const int64_t total = static_cast<int64_t>(np) * Rp;
    for (int64_t t = static_cast<int64_t>(blockIdx.x) * 256 + threadIdx.x; t < total;
         t += static_cast<int64_t>(gridDim.x) * 256) {
        const int i = static_cast<int>(t / Rp), j = static_cast<int>(t % Rp);
        const float u = (i < n && j < R) ? start_u(x0, i, R, j, sqrt_beta) : 0.0f;
        U[t] = u;
        if constexpr (PREC == 1) {
            const float m = j < R ? __uint_as_float(colmax_bits[j]) : 0.0f;
            const float c = m > 0.0f ? m / kFp8Max : 1.0f;
            if (i == 0) cs[j] = c;
            Ub[static_cast<int64_t>(j) * np + i] = to_fp8(u / c);
        } else {
            Ub[static_cast<int64_t>(j) * np + i] = to_lowp<PREC>(u);
        }
    }
}

// u -> x = u / sqrt(beta) (double) and sign(x).
__global__ __launch_bounds__(256) void lowp_finish_kernel(const float* __restrict__ U0, const float* __restrict__ U1,
                                                          const float* __restrict__ U2,
                                                          const RestartState* __restrict__ state, int n, int R,
                                                          int Rp, double sqrt_beta,
                                                          double* __restrict__ x_out,
                                                          int8_t* __restrict__ s_out) {
    const int64_t total = static_cast<int64_t>(n) * R;
    for (int64_t t = static_cast<int64_t>(blockIdx.x) * 256 + threadIdx.x; t < total;
         t += static_cast<int64_t>(gridDim.x) * 256) {
        const int i = static_cast<int>(t / R), j = static_cast<int>(t % R);
        // restart j's last iterate: buffer iters_done mod 3
        const int64_t m = state[j].iters_done % 3;
        const float* U = m == 0 ? U0 : (m == 1 ? U1 : U2);
        const double x = ddiv(static_cast<double>(U[static_cast<int64_t>(i) * Rp + j]), sqrt_beta);
        if (x_out) x_out[t] = x;
        if (s_out) s_out[t] = x >= 0.0 ? 1 : -1;
    }
}

// FP64 J -> padded BF16 copy, or FP8 copy with per-row scales and the
// absolute row sums s_i sum_j |q_ij| of the quantised rows (rowabs).
template <int PREC>
__global__ __launch_bounds__(256) void lowp_convert_kernel(const double* __restrict__ J, int n, int np,
                                                           typename Prec<PREC>::T* __restrict__ Jq,
                                                           float* __restrict__ rscale,
                                                           double* __restrict__ rowabs) {
    __shared__ double red[4];
    for (int i = blockIdx.x; i < np; i += gridDim.x) {
        float s = 1.0f;
        if (PREC == 1) {
            double m = 0.0;
            if (i < n)
                for (int c = threadIdx.x; c < n; c += 256) m = fmax(m, fabs(J[static_cast<int64_t>(i) * n + c]));
            m = wave_max(m);
            if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = m;
            __syncthreads();
            m = fmax(fmax(red[0], red[1]), fmax(red[2], red[3]));
            __syncthreads();
            s = m > 0.0 ? static_cast<float>(m / 448.0) : 1.0f;
            if (threadIdx.x == 0) rscale[i] = s;
        }
        double ra = 0.0;
        for (int c = threadIdx.x; c < np; c += 256) {
            const double v = (i < n && c < n) ? J[static_cast<int64_t>(i) * n + c] : 0.0;
            if constexpr (PREC == 1) {
                const uint8_t q = to_fp8(static_cast<float>(v / static_cast<double>(s)));
                Jq[static_cast<int64_t>(i) * np + c] = q;
                ra = dadd(ra, fabs(fp8_value(q)));
            } else {
                Jq[static_cast<int64_t>(i) * np + c] = to_lowp<PREC>(static_cast<float>(v));
            }
        }
        if constexpr (PREC == 1) {
            ra = wave_sum(ra);
            if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = ra;
            __syncthreads();
            if (threadIdx.x == 0)
                rowabs[i] = dmul(dadd(dadd(red[0], red[1]), dadd(red[2], red[3])), static_cast<double>(s));
            __syncthreads();
        }
    }
}

// FP64 objective of R final iterates with the FP64 J (eq:Hamilton).  Z = J X
// is a dense (n x n) by (n x R) FP64 product: 64 x 64 output tiles per
// workgroup, each thread a 4 x 4 block, J and X staged through LDS in k
// slices of 32, so J is read once per 64 restarts instead of once per
// restart.  The epilogue reduces x^4, x^2 and x z per restart over the tile's
// rows; the last workgroup of each column block adds the row tiles in order
// and writes H.
__global__ __launch_bounds__(256) void dense_objective_kernel(const double* __restrict__ J, int n,
                                                              int R, int Rp,
                                                              const double* __restrict__ X,
                                                              double alpha, double beta,
                                                              double* __restrict__ partials,
                                                              unsigned int* tickets,
                                                              double* __restrict__ H) {
    constexpr int KS = 32;
    __shared__ double Js[64][KS + 1];
    __shared__ double Xs[KS][64];
    __shared__ double cred[16][64][3];
    __shared__ int last_flag;
    const int tid = threadIdx.x;
    const int ty = tid >> 4, tx = tid & 15;
    const int row0 = blockIdx.x * 64, col0 = blockIdx.y * 64;
    double acc[4][4] = {};
    for (int k0 = 0; k0 < n; k0 += KS) {
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const int e = tid + 256 * u;
            const int r = e / KS, kk = e % KS;
            const int gi = row0 + r, gk = k0 + kk;
            Js[r][kk] = (gi < n && gk < n) ? J[static_cast<int64_t>(gi) * n + gk] : 0.0;
            const int xk = e / 64, xc = e % 64;
            const int hk = k0 + xk, hc = col0 + xc;
            Xs[xk][xc] = (hk < n && hc < R) ? X[static_cast<int64_t>(hk) * R + hc] : 0.0;
        }
        __syncthreads();
#pragma unroll 8
        for (int kk = 0; kk < KS; ++kk) {
            double a[4], b[4];
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                a[q] = Js[ty * 4 + q][kk];
                b[q] = Xs[kk][tx * 4 + q];
            }
#pragma unroll
            for (int p = 0; p < 4; ++p)
#pragma unroll
                for (int q = 0; q < 4; ++q) acc[p][q] = fma(a[p], b[q], acc[p][q]);
        }
        __syncthreads();
    }
    // per-column sums over this thread's 4 rows
    double v[4][3] = {};
#pragma unroll
    for (int p = 0; p < 4; ++p) {
        const int i = row0 + ty * 4 + p;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int c = col0 + tx * 4 + q;
            if (i < n && c < R) {
                const double x = X[static_cast<int64_t>(i) * R + c];
                const double x2 = dmul(x, x);
                v[q][0] = dadd(v[q][0], dmul(x2, x2));
                v[q][1] = dadd(v[q][1], x2);
                v[q][2] = dadd(v[q][2], dmul(x, acc[p][q]));
            }
        }
    }
#pragma unroll
    for (int q = 0; q < 4; ++q)
#pragma unroll
        for (int m = 0; m < 3; ++m) cred[ty][tx * 4 + q][m] = v[q][m];
    __syncthreads();
    if (tid < 64) {                             // wave 0: the wave that releases below
        double* p = partials + (static_cast<size_t>(blockIdx.x) * Rp + col0 + tid) * 3;
#pragma unroll
        for (int m = 0; m < 3; ++m) {
            double sm = 0.0;
            for (int t = 0; t < 16; ++t) sm = dadd(sm, cred[t][tid][m]);
            store_agent(p + m, sm);
        }
    }
    __syncthreads();
    if (tid == 0) last_flag = arrive_last(tickets + blockIdx.y, gridDim.x) ? 1 : 0;
    __syncthreads();
    if (!last_flag) return;
    if (tid < 3 * 64) {
        const int cl = tid & 63, m = tid >> 6;
        cred[0][cl][m] = column_partial_sum<3>(partials, Rp, col0 + cl, m, gridDim.x);
    }
    __syncthreads();
    if (tid < 64 && col0 + tid < R) {
        const double* S = cred[0][tid];
        H[col0 + tid] = dsub(dsub(dmul(ddiv(beta, 4.0), S[0]), dmul(ddiv(alpha, 2.0), S[1])), dmul(0.5, S[2]));
    }
    if (tid == 0) reset_ticket(tickets + blockIdx.y);
}

}  // namespace

hipError_t launch_lowp_convert(int prec, const double* J, int n, int np, void* Jq, float* rscale,
                               double* rowabs, hipStream_t s) {
    const int grid = np < 4096 ? np : 4096;
    if (prec == 0)
        hipLaunchKernelGGL(lowp_convert_kernel<0>, dim3(grid), dim3(256), 0, s, J, n, np,
                           static_cast<__bf16*>(Jq), rscale, rowabs);
    else
        hipLaunchKernelGGL(lowp_convert_kernel<1>, dim3(grid), dim3(256), 0, s, J, n, np,
                           static_cast<uint8_t*>(Jq), rscale, rowabs);
    return hipGetLastError();
}

hipError_t launch_lowp_load(int prec, const double* x0, int n, int R, int np, int Rp, double sqrt_beta,
                            unsigned int* colmax_bits, float* cs, float* U, void* Ub, hipStream_t s) {
    int64_t g = (static_cast<int64_t>(np) * Rp + 255) / 256;
    if (g > 8192) g = 8192;
    if (prec == 0) {
        hipLaunchKernelGGL(lowp_load_kernel<0>, dim3(static_cast<unsigned>(g)), dim3(256), 0, s, x0, n, R,
                           np, Rp, sqrt_beta, nullptr, nullptr, U, static_cast<__bf16*>(Ub));
    } else {
        hipError_t e = hipMemsetAsync(colmax_bits, 0, static_cast<size_t>(R) * sizeof(unsigned int), s);
        if (e != hipSuccess) return e;
        const dim3 cg((n + 63) / 64, (R + 255) / 256);
        hipLaunchKernelGGL(lowp_colmax_kernel, cg, dim3(256), 0, s, x0, n, R, sqrt_beta, colmax_bits);
        hipLaunchKernelGGL(lowp_load_kernel<1>, dim3(static_cast<unsigned>(g)), dim3(256), 0, s, x0, n, R,
                           np, Rp, sqrt_beta, colmax_bits, cs, U, static_cast<uint8_t*>(Ub));
    }
    return hipGetLastError();
}

bool lowp_shape_valid(int prec, int np, int Rp, const LowpShape& sh) {
    // the fused iteration (splits 0: a launch per iteration, -1: resident):
    // 64 x 64 tiles, 256-byte stages, depth 3 in BF16 only (FP8 fragments
    // leave no registers for a third stage under the two-wavefront cap)
    // (the resident kernel, which keeps more registers live, takes depth 2)
    if (sh.splits == 0 || sh.splits == -1)
        return sh.bn == 64 && sh.sb == 256 && (sh.depth == 2 || (sh.depth == 3 && prec == 0 && sh.splits == 0)) &&
               Rp % 64 == 0 && np % 64 == 0 && np * (prec == 0 ? 2 : 1) / 256 >= sh.depth;
    if (sh.splits == -2) {
        // J held in LDS: 128-row blocks, k slices of sb bytes per row (at
        // most 8 of them, the update adds their products in registers), one
        // 8-wavefront workgroup per (row block, slice); every workgroup closes
        // at most 128 restarts
        const int rowb = np * (prec == 0 ? 2 : 1);
        if (sh.bn != 128 || sh.depth != 1) return false;
        if (sh.sb != 256 && sh.sb != 512 && sh.sb != 1024) return false;
        if (np % kHeldRows != 0 || rowb % sh.sb != 0 || Rp % 64 != 0) return false;
        const int kb = rowb / sh.sb;
        const int G = np / kHeldRows * kb;
        return kb <= 8 && Rp <= 128 * G;
    }
    if (sh.bn != 64 && sh.bn != 128) return false;
    if (sh.sb != 128 && sh.sb != 256) return false;
    if (sh.depth != 2 && sh.depth != 3) return false;
    if (sh.splits != 1 && sh.splits != 2 && sh.splits != 4 && sh.splits != 8) return false;
    const int stages = np * (prec == 0 ? 2 : 1) / sh.sb;   // stages per row
    return Rp % sh.bn == 0 && np % kTileM == 0 && stages % sh.splits == 0 && stages / sh.splits >= sh.depth;
}

LowpShape lowp_default_shape(int prec, int np, int Rp, int cus) {
    // the fused iteration: no partial tiles in memory, one launch per
    // iteration (depth 3 where the padded order holds three stages in BF16)
    (void)cus;
    LowpShape sh;
    sh.bn = 64;
    sh.splits = 0;
    sh.sb = 256;
    sh.depth = 3;
    if (!lowp_shape_valid(prec, np, Rp, sh)) sh.depth = 2;
    return sh;
}

size_t lowp_product_bytes(int prec, int np, int Rp, const LowpShape& sh) {
    // the fused iteration (splits 0 or -1) keeps no partial tiles; J held in
    // LDS (splits -2) keeps one per k slice
    if (sh.splits == -2) return static_cast<size_t>(np) * (prec == 0 ? 2 : 1) / sh.sb * np * Rp * sizeof(float);
    return sh.splits > 0 ? static_cast<size_t>(sh.splits) * np * Rp * sizeof(float) : 0;
}

namespace {

struct CloseArgs {
    int64_t k;
    double alpha, beta, eps;
    const double* partials_prev;
    double* log;
    RestartState* state;
};

template <int PREC, int BN, int SB, int DEPTH>
void launch_gemm_one(dim3 g, hipStream_t s, int np, int Rp, int S, int R, const void* Jq, const void* Ub, float* P,
                     const CloseArgs& c) {
    using T = typename Prec<PREC>::T;
    if constexpr (SB == 256)
        hipLaunchKernelGGL((lowp_gemm_kernel<PREC, BN, DEPTH>), g, dim3(MT), 0, s, np, Rp, S, R,
                           static_cast<const T*>(Jq), static_cast<const T*>(Ub), P, c.k, c.alpha, c.beta, c.eps,
                           c.partials_prev, c.log, c.state);
    else
        hipLaunchKernelGGL((lowp_gemm2_kernel<PREC, BN, DEPTH>), g, dim3(MT), 0, s, np, Rp, S, R,
                           static_cast<const T*>(Jq), static_cast<const T*>(Ub), P, c.k, c.alpha, c.beta, c.eps,
                           c.partials_prev, c.log, c.state);
}

template <int PREC>
void launch_gemm(const LowpShape& sh, dim3 g, hipStream_t s, int np, int Rp, int R, const void* Jq,
                 const void* Ub, float* P, const CloseArgs& c) {
    const int key = (sh.bn == 128 ? 4 : 0) + (sh.sb == 256 ? 2 : 0) + (sh.depth == 3 ? 1 : 0);
    switch (key) {
        case 0: launch_gemm_one<PREC, 64, 128, 2>(g, s, np, Rp, sh.splits, R, Jq, Ub, P, c); break;
        case 1: launch_gemm_one<PREC, 64, 128, 3>(g, s, np, Rp, sh.splits, R, Jq, Ub, P, c); break;
        case 2: launch_gemm_one<PREC, 64, 256, 2>(g, s, np, Rp, sh.splits, R, Jq, Ub, P, c); break;
        case 3: launch_gemm_one<PREC, 64, 256, 3>(g, s, np, Rp, sh.splits, R, Jq, Ub, P, c); break;
        case 4: launch_gemm_one<PREC, 128, 128, 2>(g, s, np, Rp, sh.splits, R, Jq, Ub, P, c); break;
        case 5: launch_gemm_one<PREC, 128, 128, 3>(g, s, np, Rp, sh.splits, R, Jq, Ub, P, c); break;
        case 6: launch_gemm_one<PREC, 128, 256, 2>(g, s, np, Rp, sh.splits, R, Jq, Ub, P, c); break;
        default: launch_gemm_one<PREC, 128, 256, 3>(g, s, np, Rp, sh.splits, R, Jq, Ub, P, c); break;
    }
}

template <int PREC, int S>
void launch_update_one(dim3 g, hipStream_t s, int np, int Rp, const float* P, const float* rscale,
                       const float* U_old, float* U_new, void* Ub_new, const float* cs_old, float* cs_new,
                       double rho_q, double alpha, int R, double* partials, const RestartState* state) {
    using T = typename Prec<PREC>::T;
    hipLaunchKernelGGL((lowp_update_kernel<PREC, S>), g, dim3(MT), 0, s, np, Rp, P, rscale, U_old, U_new,
                       static_cast<T*>(Ub_new), cs_old, cs_new, rho_q, alpha, R, partials, state);
}

template <int PREC>
void launch_update(int S, dim3 g, hipStream_t s, int np, int Rp, const float* P, const float* rscale,
                   const float* U_old, float* U_new, void* Ub_new, const float* cs_old, float* cs_new,
                   double rho_q, double alpha, int R, double* partials, const RestartState* state) {
#define DOCH_LOWP_UPDATE(SS)                                                                                 \
    launch_update_one<PREC, SS>(g, s, np, Rp, P, rscale, U_old, U_new, Ub_new, cs_old, cs_new, rho_q, alpha, \
                                R, partials, state)
    switch (S) {
        case 1: DOCH_LOWP_UPDATE(1); break;
        case 2: DOCH_LOWP_UPDATE(2); break;
        case 4: DOCH_LOWP_UPDATE(4); break;
        default: DOCH_LOWP_UPDATE(8); break;
    }
#undef DOCH_LOWP_UPDATE
}

}  // namespace

hipError_t launch_lowp_step(int prec, int np, int Rp, const LowpShape& sh, const void* Jq, const float* rscale,
                            const float* U_old, float* U_new, const void* Ub_old, void* Ub_new,
                            const float* cs_old, float* cs_new, double rho_q, double alpha, double beta,
                            double eps, int R, int64_t k, float* P, const double* partials_prev,
                            double* partials, double* log, RestartState* state, hipStream_t s) {
    if (!lowp_shape_valid(prec, np, Rp, sh)) return hipErrorInvalidValue;
    if (sh.splits == 0) {
        // np / 64 row tiles per column block; the tiles close the previous
        // iteration themselves
        const dim3 grid(np / 64, Rp / 64);
#define DOCH_LOWP_FUSED(PP, DD)                                                                                 \
    hipLaunchKernelGGL((lowp_fused_kernel<PP, DD>), grid, dim3(MT), 0, s, np, Rp,                              \
                       static_cast<const Prec<PP>::T*>(Jq), rscale, U_old, U_new,                              \
                       static_cast<const Prec<PP>::T*>(Ub_old), static_cast<Prec<PP>::T*>(Ub_new), cs_old,    \
                       cs_new, rho_q, alpha, beta, eps, R, k, partials_prev, partials, log, state)
        if (prec == 0) {
            if (sh.depth == 3) DOCH_LOWP_FUSED(0, 3); else DOCH_LOWP_FUSED(0, 2);
        } else {
            DOCH_LOWP_FUSED(1, 2);
        }
#undef DOCH_LOWP_FUSED
        return hipGetLastError();
    }
    // the product tiles, then Rp / 64 workgroups closing iteration k - 1
    const dim3 pg((np / kTileM) * (Rp / sh.bn) * sh.splits + Rp / 64);
    const dim3 ug(np / 64, Rp / 64);
    const CloseArgs c{k, alpha, beta, eps, partials_prev, log, state};
    if (prec == 0) {
        launch_gemm<0>(sh, pg, s, np, Rp, R, Jq, Ub_old, P, c);
        launch_update<0>(sh.splits, ug, s, np, Rp, P, rscale, U_old, U_new, Ub_new, cs_old, cs_new, rho_q, alpha, R,
                         partials, state);
    } else {
        launch_gemm<1>(sh, pg, s, np, Rp, R, Jq, Ub_old, P, c);
        launch_update<1>(sh.splits, ug, s, np, Rp, P, rscale, U_old, U_new, Ub_new, cs_old, cs_new, rho_q, alpha, R,
                         partials, state);
    }
    return hipGetLastError();
}

namespace {

template <int PREC, int DEPTH>
hipError_t launch_resident_one(const LowpResArgs& a, hipStream_t s) {
    static int cap = 0;           // workgroups of this kernel the device holds at once
    auto kern = lowp_resident_kernel<PREC, DEPTH>;
    if (cap == 0) {
        int dev = 0, cus = 0, occ = 0;
        hipError_t e = hipGetDevice(&dev);
        if (e == hipSuccess) e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
        if (e == hipSuccess) e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, kern, MT, 0);
        if (e != hipSuccess) return e;
        cap = cus * occ;
    }
    const int groups = a.tiles * a.cblocks;
    if (groups > cap) return hipErrorCooperativeLaunchTooLarge;
    LowpResArgs arg = a;
    void* args[] = {&arg};
    return hipLaunchCooperativeKernel(reinterpret_cast<const void*>(kern), dim3(groups), dim3(MT), args, 0, s);
}

}  // namespace

hipError_t launch_lowp_resident(int prec, int np, int Rp, const LowpShape& sh, int64_t iters, const void* Jq,
                                const float* rscale, float* const* U, void* const* Ub, float* const* cs,
                                double rho_q, double alpha, double beta, double eps, int R, double* const* partials,
                                double* log, RestartState* state, ResidentSync* sync, hipStream_t s) {
    if (sh.splits != -1 || !lowp_shape_valid(prec, np, Rp, sh)) return hipErrorInvalidValue;
    LowpResArgs a{};
    a.np = np;
    a.Rp = Rp;
    a.R = R;
    a.tiles = np / 64;
    a.cblocks = Rp / 64;
    a.iters = iters;
    a.Jq = Jq;
    a.rscale = rscale;
    for (int i = 0; i < 3; ++i) {
        a.U[i] = U[i];
        a.Ub[i] = Ub[i];
        a.cs[i] = cs[i];
    }
    a.rho_q = rho_q;
    a.alpha = alpha;
    a.beta = beta;
    a.eps = eps;
    a.partials[0] = partials[0];
    a.partials[1] = partials[1];
    a.log = log;
    a.state = state;
    a.sync = sync;
    if (prec == 0) return launch_resident_one<0, 2>(a, s);
    return launch_resident_one<1, 2>(a, s);
}

namespace {

template <int PREC, int NG>
hipError_t launch_held_one(const LowpHeldArgs& a, hipStream_t s) {
    static int cap = 0;           // workgroups of this kernel the device holds at once
    auto kern = lowp_held_kernel<PREC, NG>;
    if (cap == 0) {
        int dev = 0, cus = 0, occ = 0;
        hipError_t e = hipGetDevice(&dev);
        if (e == hipSuccess) e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
        if (e == hipSuccess) e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, kern, HT, 0);
        if (e != hipSuccess) return e;
        cap = cus * occ;
    }
    const int groups = a.rblocks * a.kslices;
    if (groups > cap) return hipErrorCooperativeLaunchTooLarge;
    LowpHeldArgs arg = a;
    void* args[] = {&arg};
    return hipLaunchCooperativeKernel(reinterpret_cast<const void*>(kern), dim3(groups), dim3(HT), args, 0, s);
}

}  // namespace

hipError_t launch_lowp_held(int prec, int np, int Rp, const LowpShape& sh, int64_t iters, const void* Jq,
                            const float* rscale, float* const* U, void* const* Ub, float* const* cs, double rho_q,
                            double alpha, double beta, double eps, int R, float* P, double* const* partials,
                            double* log, RestartState* state, ResidentSync* sync, hipStream_t s) {
    if (sh.splits != -2 || !lowp_shape_valid(prec, np, Rp, sh)) return hipErrorInvalidValue;
    LowpHeldArgs a{};
    a.np = np;
    a.Rp = Rp;
    a.R = R;
    a.rblocks = np / kHeldRows;
    a.kslices = np * (prec == 0 ? 2 : 1) / sh.sb;
    a.iters = iters;
    a.Jq = Jq;
    a.rscale = rscale;
    for (int i = 0; i < 3; ++i) {
        a.U[i] = U[i];
        a.Ub[i] = Ub[i];
        a.cs[i] = cs[i];
    }
    a.rho_q = rho_q;
    a.alpha = alpha;
    a.beta = beta;
    a.eps = eps;
    a.P = P;
    a.partials[0] = partials[0];
    a.partials[1] = partials[1];
    a.log = log;
    a.state = state;
    a.sync = sync;
    const int ng = sh.sb / 128;
    if (prec == 0) {
        if (ng == 2) return launch_held_one<0, 2>(a, s);
        if (ng == 4) return launch_held_one<0, 4>(a, s);
        return launch_held_one<0, 8>(a, s);
    }
    if (ng == 2) return launch_held_one<1, 2>(a, s);
    if (ng == 4) return launch_held_one<1, 4>(a, s);
    return launch_held_one<1, 8>(a, s);
}

hipError_t launch_lowp_close(int np, int Rp, int R, int64_t kk, const double* partials, double alpha,
                             double beta, double eps, double* log, RestartState* state, hipStream_t s) {
    hipLaunchKernelGGL(lowp_close_kernel, dim3(Rp / 64), dim3(MT), 0, s, partials, np / 64, Rp, R, kk, alpha,
                       beta, eps, log, state);
    return hipGetLastError();
}

hipError_t launch_lowp_finish(const float* const* U, const RestartState* state, int n, int R, int Rp,
                              double sqrt_beta, double* x_out, int8_t* s_out, hipStream_t s) {
    int64_t g = (static_cast<int64_t>(n) * R + 255) / 256;
    if (g > 8192) g = 8192;
    hipLaunchKernelGGL(lowp_finish_kernel, dim3(static_cast<unsigned>(g)), dim3(256), 0, s, U[0], U[1], U[2],
                       state, n, R, Rp, sqrt_beta, x_out, s_out);
    return hipGetLastError();
}

hipError_t launch_dense_objective(const double* J, int n, int R, const double* X, double alpha,
                                  double beta, double* partials, unsigned int* tickets, double* H,
                                  hipStream_t s) {
    const int Rp = (R + 63) / 64 * 64;
    hipLaunchKernelGGL(dense_objective_kernel, dim3((n + 63) / 64, Rp / 64), dim3(256), 0, s, J, n, R, Rp, X,
                       alpha, beta, partials, tickets, H);
    return hipGetLastError();
}

}  // namespace doch
