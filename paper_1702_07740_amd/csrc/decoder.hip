// Flooding sum-product decoding of QC LDPC codes in syndrome form, gfx950.
//
// One decode is a short sequence of launches on the caller's stream:
//   init      fail flags, packed syndrome bits, core totals L = Q, and the
//             degree-1 inputs Psi = +-Phi(|Q|)
//   t = 1..T  check pass (Alg. 1 Step 2, plus the Step 4 check of iteration
//             t-1) and variable pass (Step 3, core columns)
//   vote      the Step 4 check of the last iteration
//   finalize  hard decisions, posteriors, iteration counts
//
// Edge state.  Messages live per non-zero base block as one array of Z values
// in check order: block (r, c) with shift s holds m(r*Z + a -> c*Z + (a+s)%Z)
// at index a.  The check pass reads and writes each array contiguously; the
// variable pass reads block (r, c) at index (j - s) mod Z, contiguous with one
// wrap.  No index arrays exist: the circulant shift is the whole addressing.
//
// Degree-1 columns (the long diagonal, Sec. III-C) keep no state: their
// variable-to-check message is the constant channel LLR Q, so Phi(|Q|) is
// evaluated once per decode (Psi, stored in check order with the sign of Q).
// Their posterior Q + m is needed only for the decision bit, and its sign
// follows from the Phi domain without evaluating m: Phi is a decreasing
// involution, so |Q| > |m| = Phi(S) exactly when Phi(|Q|) < S, where S is the
// exclusive Phi sum of the check's other inputs.  The decision bits are stored
// packed by check position (one bit per degree-1 block and check).
//
// Early stop.  Frame f's check for iteration t-1 is evaluated inside check
// pass t from values that pass gathers anyway (core totals of iteration t-1 and
// degree-1 decision bits of iteration t-1), and written to fail[t-1][f].  Every
// pass skips a frame whose earlier check succeeded; the variable pass t skips
// a frame whose check at t-1 succeeded, so the frame's totals and degree-1 bits
// stay those of its exit iteration.
//
// Addressing.  Every array is reached from a workgroup-uniform base pointer
// plus a 32-bit lane offset, so loads and stores use the scalar-base form.
#include "internal.h"

#include <hip/hip_fp16.h>

namespace ldpc {

namespace {

constexpr int kBlock = 256;  // threads per workgroup: 4 wave64s
constexpr float kPhiLo = 1e-7f;
constexpr float kPhiHi = 30.0f;

// Phi(x) = -ln tanh(x/2) on the clamped argument [1e-7, 30], branch-free:
//   x <  2: Phi(x) = ln 2 - ln x + g(x^2/4), where g(u) = -ln(tanh(y)/y),
//           y = sqrt(u), is smooth and even; g(w/4) = w H(w) with H a degree-6
//           least-squares fit on [0, 4] (absolute error 3e-9);
//   x >= 2: Phi(x) = 2 atanh(t), t = e^{-x} <= 0.136, by its odd series to t^9
//           (truncation below 3e-10 relative; no cancellation for large x).
// Both branches use one hardware transcendental (log2 or exp2).  Relative
// error below 1e-6 for x < 20 and below 2e-6 up to 30 (there Phi < 2e-9).
__device__ __forceinline__ float phi_f32(float x) {
    constexpr float kLog2e = 1.4426950408889634f;
    constexpr float kLn2 = 0.6931471805599453f;
    x = __builtin_amdgcn_fmed3f(x, kPhiLo, kPhiHi);
    const float w = x * x;
    float h = 5.28133137e-09f;
    h = fmaf(w, h, -1.35732463e-07f);
    h = fmaf(w, h, 2.02647516e-06f);
    h = fmaf(w, h, -2.61091045e-05f);
    h = fmaf(w, h, 3.41622334e-04f);
    h = fmaf(w, h, -4.86108987e-03f);
    h = fmaf(w, h, 8.33333358e-02f);
    const float small = fmaf(-kLn2, __builtin_amdgcn_logf(x), kLn2) + w * h;
    const float t = __builtin_amdgcn_exp2f(-x * kLog2e);
    const float t2 = t * t;
    float p = fmaf(t2, 2.0f / 9.0f, 2.0f / 7.0f);
    p = fmaf(t2, p, 2.0f / 5.0f);
    p = fmaf(t2, p, 2.0f / 3.0f);
    p = fmaf(t2, p, 2.0f);
    const float large = t * p;
    return x < 2.0f ? small : large;
}

template <typename Msg> __device__ __forceinline__ float msg_load(const Msg *p);
template <> __device__ __forceinline__ float msg_load<float>(const float *p) { return *p; }
template <> __device__ __forceinline__ float msg_load<_Float16>(const _Float16 *p) {
    return static_cast<float>(*p);
}
template <typename Msg> __device__ __forceinline__ void msg_store(Msg *p, float v);
template <> __device__ __forceinline__ void msg_store<float>(float *p, float v) { *p = v; }
template <> __device__ __forceinline__ void msg_store<_Float16>(_Float16 *p, float v) {
    *p = static_cast<_Float16>(v);
}

__device__ __forceinline__ unsigned long long wave_ballot(bool p) { return __ballot(p); }

// Element idx of an array, with the byte offset formed in 32-bit arithmetic so
// the access uses a uniform 64-bit base plus a 32-bit lane offset.  Every
// per-frame array here is far below 4 GB.
template <typename T>
__device__ __forceinline__ T &at(T *base, unsigned idx) {
    return *reinterpret_cast<T *>(reinterpret_cast<char *>(base) + idx * (unsigned)sizeof(T));
}
template <typename T>
__device__ __forceinline__ const T &at(const T *base, unsigned idx) {
    return *reinterpret_cast<const T *>(reinterpret_cast<const char *>(base) +
                                        idx * (unsigned)sizeof(T));
}

struct CnArgs {
    const float *llr;          // [F][n]
    const float *psi;          // [F][ND1][Z] +-Phi(|Q|) of degree-1 variables, check order
    void *msg;                 // [F][NS][Z] messages (float or half)
    const float *tot;          // [F][NC][Z] core totals of iteration t-1
    const uint64_t *d1_prev;   // [F][ND1][W] degree-1 decision bits of iteration t-1
    uint64_t *d1_cur;          // [F][ND1][W] degree-1 decision bits of iteration t
    const uint64_t *synbits;   // [F][mb][W]
    int32_t *fail;             // [T+1][F]
    float *d1post;             // [F][ND1][Z] degree-1 posteriors of iteration t, or null
    size_t msg_frame, tot_frame, d1_frame, syn_frame, psi_frame;
    int F, t;
    int update;                // 1: compute the messages of iteration t
    int first;                 // 1: t == 1, all stored messages are zero
    int vote;                  // 1: evaluate the check of iteration t-1 (or t, vote-only)
    int d1_from_llr;           // 1: the voted iteration is 0, decisions come from Q
    int skip_after;            // frame inactive if fail[skip_after][f] == 0 (-1: never)
};

// Workgroup-uniform view of one base row of one frame.
template <int D, typename Msg>
struct RowCtx {
    const float *tot;         // frame's core totals
    Msg *msg;                 // frame's messages
    const float *psi;         // frame's degree-1 inputs
    const float *llr;         // frame's channel LLRs
    const uint64_t *d1_prev;  // frame's decision bits of iteration t-1
    uint64_t *d1_cur;         // frame's decision bits of iteration t
    float *d1post;            // frame's degree-1 posteriors (or null)
    const uint64_t *syn;      // this row's packed syndrome words
    unsigned shift[D];        // circulant shift of each block
    unsigned off[D];          // state: msg offset ref*Z; degree-1: psi offset ref*Z
    unsigned src[D];          // state: totals offset core*Z; degree-1: llr offset col*Z
    unsigned wrd[D];          // degree-1: decision-word offset ref*W
    int ns;                   // blocks 0..ns-1 keep stored messages, the rest are degree-1
    unsigned Z, W;
};

template <int D, typename Msg>
__device__ __forceinline__ RowCtx<D, Msg> load_row(const CodeDev &c, const CnArgs &A, int f,
                                                   int r) {
    RowCtx<D, Msg> R;
    const unsigned Z = (unsigned)c.Z;
    R.Z = Z;
    R.W = (unsigned)c.W;
    R.tot = A.tot + (size_t)f * A.tot_frame;
    R.msg = reinterpret_cast<Msg *>(A.msg) + (size_t)f * A.msg_frame;
    R.psi = A.psi + (size_t)f * A.psi_frame;
    R.llr = A.llr + (size_t)f * c.n;
    R.d1_prev = A.d1_prev + (size_t)f * A.d1_frame;
    R.d1_cur = A.d1_cur ? A.d1_cur + (size_t)f * A.d1_frame : nullptr;
    R.d1post = A.d1post ? A.d1post + (size_t)f * A.psi_frame : nullptr;
    R.syn = A.synbits + (size_t)f * A.syn_frame + (size_t)r * c.W;
    const int b0 = c.row_first[r];
    R.ns = c.row_ns[r];
#pragma unroll
    for (int k = 0; k < D; ++k) {
        const int b = b0 + k;
        const bool st = k < R.ns;
        const unsigned ref = (unsigned)c.blk_ref[b];
        R.shift[k] = (unsigned)c.blk_shift[b];
        R.off[k] = ref * Z;
        R.src[k] = (unsigned)(st ? c.blk_core[b] : c.blk_col[b]) * Z;
        R.wrd[k] = ref * R.W;
    }
    return R;
}

// Is block k of a row with DS stored blocks a stored block?  DS >= 0 is known
// at compile time; DS < 0 reads the row's count.
template <int DS, int D, typename Msg>
__device__ __forceinline__ bool stored(const RowCtx<D, Msg> &R, int k) {
    if constexpr (DS >= 0) return k < DS;
    else return k < R.ns;
}

// Checks per thread: a thread handles checks a, a + 256, a + 512, a + 768 of
// one row, so the row's table reads are paid once and every thread has its
// loads for several checks in flight together.
constexpr int kChecksPerThread = 4;
// how many of those are processed at once (bounded by registers for large D)
template <int D> struct ChunkOf { static constexpr int value = D <= 4 ? 2 : 1; };

// K checks (r, a_first + q*256), q < K, of one frame, row degree D.  Padding
// lanes (a >= Z) take part in the wave ballots with zero bits and touch no
// memory.  Returns 1 if one of this thread's checks fails the parity check of
// the voted iteration.
template <int D, int DS, int K, typename Msg>
__device__ __forceinline__ int check_chunk(const RowCtx<D, Msg> &R, const CnArgs &A,
                                           unsigned a_first) {
    const unsigned Z = R.Z;
    const bool read_old = A.update && !A.first;

    float x[K][D];   // inputs L_vc of iteration t-1 (degree-1: Psi)
    int vpar[K];     // parity of the voted decisions on each check, with s_c
    int sb[K];       // syndrome bits
#pragma unroll
    for (int q = 0; q < K; ++q) {
        const unsigned a = a_first + q * kBlock;
        const bool valid = a < Z;
        const unsigned w = a >> 6, bit = a & 63u;
        sb[q] = valid ? (int)((at(R.syn, w) >> bit) & 1ull) : 0;
        int par = 0;
#pragma unroll
        for (int k = 0; k < D; ++k) {
            unsigned j = a + R.shift[k];
            j -= (j >= Z) ? Z : 0u;
            float xv = 1.0f;
            int dec = 0;
            if (stored<DS>(R, k)) {
                if (valid) {
                    const float lt = at(R.tot, R.src[k] + j);
                    dec = lt < 0.0f;
                    const float mo = read_old ? msg_load<Msg>(&at(R.msg, R.off[k] + a)) : 0.0f;
                    xv = lt - mo;
                }
            } else if (valid) {
                xv = at(R.psi, R.off[k] + a);
                if (A.vote)
                    dec = A.d1_from_llr ? (xv < 0.0f)
                                        : (int)((at(R.d1_prev, R.wrd[k] + w) >> bit) & 1ull);
            }
            x[q][k] = xv;
            par ^= dec;
        }
        vpar[q] = valid ? (par ^ sb[q]) : 0;
    }
    int bad = 0;
    if (A.vote) {
#pragma unroll
        for (int q = 0; q < K; ++q) bad |= vpar[q];
    }
    if (!A.update) return bad;

#pragma unroll
    for (int q = 0; q < K; ++q) {
        const unsigned a = a_first + q * kBlock;
        const bool valid = a < Z;
        const unsigned w = a >> 6;
        // Step 2: sign product with the syndrome bit, Phi-domain exclusive sums
        float ph[D];
        int neg = 0, par = sb[q];
#pragma unroll
        for (int k = 0; k < D; ++k) {
            const int nk = x[q][k] < 0.0f;
            neg |= nk << k;
            par ^= nk;
            ph[k] = stored<DS>(R, k) ? phi_f32(fabsf(x[q][k])) : fabsf(x[q][k]);
        }
        float pre[D];
        pre[0] = 0.0f;
#pragma unroll
        for (int k = 1; k < D; ++k) pre[k] = pre[k - 1] + ph[k - 1];
        float ex[D];
        float suf = 0.0f;
#pragma unroll
        for (int k = D - 1; k >= 0; --k) {
            ex[k] = pre[k] + suf;
            suf += ph[k];
        }
#pragma unroll
        for (int k = 0; k < D; ++k) {
            const int sgn = (par ^ (neg >> k)) & 1;  // 1: the message to block k is negative
            if (stored<DS>(R, k)) {
                const float mag = phi_f32(ex[k]);
                if (valid) msg_store<Msg>(&at(R.msg, R.off[k] + a), sgn ? -mag : mag);
            } else {
                // decision of the degree-1 variable: sign of Q + m
                const int negq = (neg >> k) & 1;
                const float S = __builtin_amdgcn_fmed3f(ex[k], kPhiLo, kPhiHi);
                const int dec = (negq == sgn) ? negq : (ph[k] < S ? negq : sgn);
                const unsigned long long bits = wave_ballot(valid && dec);
                if ((threadIdx.x & 63) == 0 && valid) at(R.d1_cur, R.wrd[k] + w) = bits;
                if (R.d1post && valid) {
                    unsigned j = a + R.shift[k];
                    j -= (j >= Z) ? Z : 0u;
                    const float mag = phi_f32(ex[k]);
                    at(R.d1post, R.off[k] + a) = at(R.llr, R.src[k] + j) + (sgn ? -mag : mag);
                }
            }
        }
    }
    return bad;
}

template <int D, int DS, typename Msg>
__device__ __forceinline__ void check_row(const CodeDev &c, const CnArgs &A, int f, int r) {
    const RowCtx<D, Msg> R = load_row<D, Msg>(c, A, f, r);
    constexpr int K = ChunkOf<D>::value;
    const unsigned a0 = blockIdx.x * (kBlock * kChecksPerThread) + threadIdx.x;
    int bad = 0;
#pragma unroll
    for (int q0 = 0; q0 < kChecksPerThread; q0 += K)
        bad |= check_chunk<D, DS, K, Msg>(R, A, a0 + q0 * kBlock);
    if (A.vote) {
        // One flag per frame and iteration, set by any workgroup holding an
        // unsatisfied check.  Every writer stores the same value, so plain
        // stores suffice; reading first keeps all but a few workgroups per
        // frame from storing at all (the next launch sees the stores).
        bad = __syncthreads_or(bad);
        if (bad && threadIdx.x == 0) {
            int32_t *flag = A.fail + (size_t)(A.update ? A.t - 1 : A.t) * A.F + f;
            if (*reinterpret_cast<volatile int32_t *>(flag) == 0) *flag = 1;
        }
    }
}

// One launch covers the rows of one degree class; grid.y walks that class's
// rows in the row list.  Small rows are compiled for every (degree, stored
// blocks) pair, large rows for every degree with the split read at run time.
template <typename Msg, bool kLarge>
__global__ __launch_bounds__(kBlock) void check_pass(CodeDev c, CnArgs A) {
    const int f = blockIdx.z;
    const int r = c.row_list[(kLarge ? c.n_small : 0) + (int)blockIdx.y];
    if (A.skip_after >= 0 && A.fail[(size_t)A.skip_after * A.F + f] == 0) return;
#define LDPC_CASE(D) \
    case D: check_row<D, -1, Msg>(c, A, f, r); break;
#define LDPC_CASE2(D, S) \
    case (D) * 32 + (S): check_row<D, S, Msg>(c, A, f, r); break;
    if (!kLarge) {
        static_assert(kSmallRowDegree == 6, "case list below covers degrees 1..6");
        switch (c.row_deg[r] * 32 + c.row_ns[r]) {
            LDPC_CASE2(1, 0) LDPC_CASE2(1, 1)
            LDPC_CASE2(2, 0) LDPC_CASE2(2, 1) LDPC_CASE2(2, 2)
            LDPC_CASE2(3, 0) LDPC_CASE2(3, 1) LDPC_CASE2(3, 2) LDPC_CASE2(3, 3)
            LDPC_CASE2(4, 0) LDPC_CASE2(4, 1) LDPC_CASE2(4, 2) LDPC_CASE2(4, 3) LDPC_CASE2(4, 4)
            LDPC_CASE2(5, 0) LDPC_CASE2(5, 1) LDPC_CASE2(5, 2) LDPC_CASE2(5, 3) LDPC_CASE2(5, 4)
            LDPC_CASE2(5, 5)
            LDPC_CASE2(6, 0) LDPC_CASE2(6, 1) LDPC_CASE2(6, 2) LDPC_CASE2(6, 3) LDPC_CASE2(6, 4)
            LDPC_CASE2(6, 5) LDPC_CASE2(6, 6)
            default: break;
        }
    } else {
        static_assert(LDPC_MAX_ROW_DEGREE == 16, "case list below covers degrees 7..16");
        switch (c.row_deg[r]) {
            LDPC_CASE(7) LDPC_CASE(8) LDPC_CASE(9) LDPC_CASE(10) LDPC_CASE(11) LDPC_CASE(12)
            LDPC_CASE(13) LDPC_CASE(14) LDPC_CASE(15) LDPC_CASE(16)
            default: break;
        }
    }
#undef LDPC_CASE
#undef LDPC_CASE2
}

template <typename Msg>
void launch_check_pass(const CodeDev &c, const CnArgs &a, int F, hipStream_t st) {
    const unsigned tiles_a =
        (unsigned)((c.Z + kBlock * kChecksPerThread - 1) / (kBlock * kChecksPerThread));
    if (c.n_small > 0)
        check_pass<Msg, false><<<dim3(tiles_a, c.n_small, F), dim3(kBlock), 0, st>>>(c, a);
    if (c.n_large > 0)
        check_pass<Msg, true><<<dim3(tiles_a, c.n_large, F), dim3(kBlock), 0, st>>>(c, a);
}

struct VnArgs {
    const float *llr;
    const void *msg;
    float *tot;
    const int32_t *fail;
    size_t msg_frame, tot_frame;
    int F, t;
};

// Step 3 for the core columns: L_v = Q_v + sum of the column's messages, in
// increasing row order.  One thread per (core column, position j).
template <typename Msg>
__global__ __launch_bounds__(kBlock) void variable_pass(CodeDev c, VnArgs A) {
    const int f = blockIdx.z;
    const int k = blockIdx.y;
    if (A.fail[(size_t)(A.t - 1) * A.F + f] == 0) return;
    const unsigned Z = (unsigned)c.Z;
    const unsigned j = blockIdx.x * kBlock + threadIdx.x;
    if (j >= Z) return;
    const Msg *msg = reinterpret_cast<const Msg *>(A.msg) + (size_t)f * A.msg_frame;
    const float *llr = A.llr + (size_t)f * c.n + (size_t)c.core_col[k] * Z;
    float L = llr[j];
    const int i0 = c.core_first[k], deg = c.core_deg[k];
    // loads issued 16 at a time, sums kept in increasing row order
    constexpr int U = 16;
    int i = 0;
    for (; i + U <= deg; i += U) {
        float v[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const unsigned s = (unsigned)c.core_shift[i0 + i + u];
            const unsigned idx = (j >= s) ? j - s : j + Z - s;
            v[u] = msg_load<Msg>(msg + (unsigned)c.core_state[i0 + i + u] * Z + idx);
        }
#pragma unroll
        for (int u = 0; u < U; ++u) L += v[u];
    }
    for (; i < deg; ++i) {
        const unsigned s = (unsigned)c.core_shift[i0 + i];
        const unsigned idx = (j >= s) ? j - s : j + Z - s;
        L += msg_load<Msg>(msg + (unsigned)c.core_state[i0 + i] * Z + idx);
    }
    A.tot[(size_t)f * A.tot_frame + (size_t)k * Z + j] = L;
}

// fail[t][f] = 1 marks "iteration t not checked or check failed".
__global__ void init_fail(int32_t *fail, int F, int T, int early_stop, int check_from) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= (T + 1) * F) return;
    const int t = i / F;
    const bool checked = (t == T) || (early_stop && t >= check_from);
    fail[i] = checked ? 0 : 1;
}

// Pack the syndrome bytes into 64-bit words per base row: bit a%64 of word a/64.
__global__ __launch_bounds__(kBlock) void pack_syndrome(CodeDev c, const uint8_t *syn,
                                                        uint64_t *synbits, size_t syn_frame) {
    const int f = blockIdx.z, r = blockIdx.y;
    const int a = blockIdx.x * kBlock + threadIdx.x;
    const bool valid = a < c.Z;
    const int v = valid ? (syn[(size_t)f * c.m + (size_t)r * c.Z + a] & 1) : 0;
    const unsigned long long bits = wave_ballot(v != 0);
    if ((threadIdx.x & 63) == 0 && valid)
        synbits[(size_t)f * syn_frame + (size_t)r * c.W + (a >> 6)] = bits;
}

// Core totals of iteration 0: L_v = Q_v.
__global__ __launch_bounds__(kBlock) void init_totals(CodeDev c, const float *llr, float *tot,
                                                      size_t tot_frame) {
    const int f = blockIdx.z, k = blockIdx.y;
    const int j = blockIdx.x * kBlock + threadIdx.x;
    if (j >= c.Z) return;
    tot[(size_t)f * tot_frame + (size_t)k * c.Z + j] =
        llr[(size_t)f * c.n + (size_t)c.core_col[k] * c.Z + j];
}

// Degree-1 inputs in check order: Psi[a] = +-Phi(|Q_p|), p the variable of
// check a of degree-1 block k, with the sign of Q_p (negative iff Q_p < 0).
__global__ __launch_bounds__(kBlock) void init_psi(CodeDev c, const float *llr, float *psi,
                                                   size_t psi_frame) {
    const int f = blockIdx.z, k = blockIdx.y;
    const unsigned Z = (unsigned)c.Z;
    const unsigned a = blockIdx.x * kBlock + threadIdx.x;
    if (a >= Z) return;
    unsigned j = a + (unsigned)c.d1_shift[k];
    j -= (j >= Z) ? Z : 0u;
    const float q = llr[(size_t)f * c.n + (size_t)c.d1_col[k] * Z + j];
    const float p = phi_f32(fabsf(q));
    psi[(size_t)f * psi_frame + (size_t)k * Z + a] = q < 0.0f ? -p : p;
}

struct FinArgs {
    const float *llr;
    const float *tot;
    const uint64_t *d1bits[2];
    const float *d1post[2];
    const int32_t *fail;
    uint8_t *bits_out;
    int32_t *iters_out;
    uint8_t *conv_out;
    float *llr_out;
    size_t tot_frame, d1_frame, psi_frame;
    int F, T;
};

__global__ __launch_bounds__(kBlock) void finalize(CodeDev c, FinArgs A) {
    const int f = blockIdx.y;
    int it = A.T, conv = 0;
    for (int t = 0; t <= A.T; ++t)
        if (A.fail[(size_t)t * A.F + f] == 0) {
            it = t;
            conv = 1;
            break;
        }
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        A.iters_out[f] = it;
        A.conv_out[f] = (uint8_t)conv;
    }
    const int v = blockIdx.x * kBlock + threadIdx.x;
    if (v >= c.n) return;
    const int Z = c.Z;
    const int col = v / Z;
    const int j = v - col * Z;
    const int kind = c.col_kind[col], ref = c.col_ref[col];
    const float q = A.llr[(size_t)f * c.n + v];
    float L = q;
    int bit = q < 0.0f;
    if (kind == COL_CORE) {
        L = A.tot[(size_t)f * A.tot_frame + (size_t)ref * Z + j];
        bit = L < 0.0f;
    } else if (kind == COL_DEG1 && it > 0) {
        int a = j - c.d1_shift[ref];
        a += (a < 0) ? Z : 0;
        const uint64_t wd = A.d1bits[it & 1][(size_t)f * A.d1_frame + (size_t)ref * c.W + (a >> 6)];
        bit = (int)((wd >> (a & 63)) & 1ull);
        if (A.llr_out) L = A.d1post[it & 1][(size_t)f * A.psi_frame + (size_t)ref * Z + a];
    }
    A.bits_out[(size_t)f * c.n + v] = (uint8_t)bit;
    if (A.llr_out) A.llr_out[(size_t)f * c.n + v] = L;
}

__global__ __launch_bounds__(kBlock) void syndrome_kernel(CodeDev c, const uint8_t *bits,
                                                          uint8_t *syn) {
    const int f = blockIdx.z, r = blockIdx.y;
    const int a = blockIdx.x * kBlock + threadIdx.x;
    if (a >= c.Z) return;
    const uint8_t *x = bits + (size_t)f * c.n;
    const int b0 = c.row_first[r], d = c.row_deg[r];
    int p = 0;
    for (int k = 0; k < d; ++k) {
        int j = a + c.blk_shift[b0 + k];
        j -= (j >= c.Z) ? c.Z : 0;
        p ^= x[(size_t)c.blk_col[b0 + k] * c.Z + j] & 1;
    }
    syn[(size_t)f * c.m + (size_t)r * c.Z + a] = (uint8_t)p;
}

inline size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }
inline unsigned tiles(int n) { return (unsigned)((n + kBlock - 1) / kBlock); }

template <typename Msg>
hipError_t enqueue_typed(const DecodeLaunch &l, const WorkLayout &L) {
    const CodeDev &c = l.c;
    const int F = l.F, T = l.T;
    char *ws = l.ws;
    void *msg = ws + L.msg;
    float *tot = reinterpret_cast<float *>(ws + L.tot);
    float *psi = reinterpret_cast<float *>(ws + L.psi);
    uint64_t *d1b[2] = {reinterpret_cast<uint64_t *>(ws + L.d1bits),
                        reinterpret_cast<uint64_t *>(ws + L.d1bits) + (size_t)F * L.d1bits_frame};
    uint64_t *synbits = reinterpret_cast<uint64_t *>(ws + L.synbits);
    int32_t *fail = reinterpret_cast<int32_t *>(ws + L.fail);
    float *d1p[2] = {nullptr, nullptr};
    if (l.llr_out) {
        d1p[0] = reinterpret_cast<float *>(ws + L.d1post);
        d1p[1] = d1p[0] + (size_t)F * L.psi_frame;
    }
    hipStream_t st = l.stream;

    const int nfail = (T + 1) * F;
    init_fail<<<dim3((nfail + kBlock - 1) / kBlock), dim3(kBlock), 0, st>>>(fail, F, T, l.early_stop,
                                                                           l.check_from);
    pack_syndrome<<<dim3(tiles(c.Z), c.mb, F), dim3(kBlock), 0, st>>>(c, l.syndrome, synbits,
                                                                     L.synbits_frame);
    if (c.NC > 0)
        init_totals<<<dim3(tiles(c.Z), c.NC, F), dim3(kBlock), 0, st>>>(c, l.llr, tot, L.tot_frame);
    if (c.ND1 > 0)
        init_psi<<<dim3(tiles(c.Z), c.ND1, F), dim3(kBlock), 0, st>>>(c, l.llr, psi, L.psi_frame);

    auto checked = [&](int t) { return t == T || (l.early_stop && t >= l.check_from); };

    CnArgs a{};
    a.llr = l.llr;
    a.psi = psi;
    a.msg = msg;
    a.tot = tot;
    a.synbits = synbits;
    a.fail = fail;
    a.msg_frame = L.msg_frame;
    a.tot_frame = L.tot_frame;
    a.d1_frame = L.d1bits_frame;
    a.syn_frame = L.synbits_frame;
    a.psi_frame = L.psi_frame;
    a.F = F;

    VnArgs v{};
    v.llr = l.llr;
    v.msg = msg;
    v.tot = tot;
    v.fail = fail;
    v.msg_frame = L.msg_frame;
    v.tot_frame = L.tot_frame;
    v.F = F;
    const dim3 vn_grid(tiles(c.Z), c.NC, F);

    for (int t = 1; t <= T; ++t) {
        a.t = t;
        a.update = 1;
        a.first = (t == 1);
        a.vote = checked(t - 1) ? 1 : 0;
        a.d1_from_llr = (t == 1);
        a.d1_prev = d1b[(t - 1) & 1];
        a.d1_cur = d1b[t & 1];
        a.d1post = d1p[t & 1];
        a.skip_after = t >= 2 ? t - 2 : -1;
        if (l.events) (void)hipEventRecord(l.events[2 * (t - 1)], st);
        launch_check_pass<Msg>(c, a, F, st);
        if (l.events) (void)hipEventRecord(l.events[2 * (t - 1) + 1], st);
        if (c.NC > 0) {
            v.t = t;
            variable_pass<Msg><<<vn_grid, dim3(kBlock), 0, st>>>(c, v);
        }
    }
    if (l.events) (void)hipEventRecord(l.events[2 * T], st);
    // the check of the last iteration (or of the channel decisions when T = 0)
    a.t = T;
    a.update = 0;
    a.first = 0;
    a.vote = 1;
    a.d1_from_llr = (T == 0);
    a.d1_prev = d1b[T & 1];
    a.d1_cur = nullptr;
    a.d1post = nullptr;
    a.skip_after = T >= 1 ? T - 1 : -1;
    launch_check_pass<Msg>(c, a, F, st);

    FinArgs fa{};
    fa.llr = l.llr;
    fa.tot = tot;
    fa.d1bits[0] = d1b[0];
    fa.d1bits[1] = d1b[1];
    fa.d1post[0] = d1p[0];
    fa.d1post[1] = d1p[1];
    fa.fail = fail;
    fa.bits_out = l.bits_out;
    fa.iters_out = l.iters_out;
    fa.conv_out = l.conv_out;
    fa.llr_out = l.llr_out;
    fa.tot_frame = L.tot_frame;
    fa.d1_frame = L.d1bits_frame;
    fa.psi_frame = L.psi_frame;
    fa.F = F;
    fa.T = T;
    finalize<<<dim3(tiles(c.n), F), dim3(kBlock), 0, st>>>(c, fa);
    return hipGetLastError();
}

}  // namespace

WorkLayout work_layout(const CodeDev &c, int F, int T, bool fp16, bool want_llr) {
    WorkLayout L{};
    const size_t Z = (size_t)c.Z;
    L.msg_frame = (size_t)c.NS * Z;
    L.tot_frame = (size_t)c.NC * Z;
    L.d1bits_frame = (size_t)c.ND1 * c.W;
    L.synbits_frame = (size_t)c.mb * c.W;
    L.psi_frame = (size_t)c.ND1 * Z;
    size_t off = 0;
    L.msg = off;
    off = align256(off + (size_t)F * L.msg_frame * (fp16 ? 2 : 4));
    L.tot = off;
    off = align256(off + (size_t)F * L.tot_frame * 4);
    L.psi = off;
    off = align256(off + (size_t)F * L.psi_frame * 4);
    L.d1bits = off;
    off = align256(off + 2 * (size_t)F * L.d1bits_frame * 8);
    L.synbits = off;
    off = align256(off + (size_t)F * L.synbits_frame * 8);
    L.fail = off;
    off = align256(off + (size_t)(T + 1) * F * 4);
    L.d1post = off;
    if (want_llr) off = align256(off + 2 * (size_t)F * L.psi_frame * 4);
    L.total = off;
    return L;
}

hipError_t enqueue_decode(const DecodeLaunch &l) {
    const WorkLayout L = work_layout(l.c, l.F, l.T, l.fp16 != 0, l.llr_out != nullptr);
    return l.fp16 ? enqueue_typed<_Float16>(l, L) : enqueue_typed<float>(l, L);
}

hipError_t enqueue_syndrome(const CodeDev &c, int F, const uint8_t *bits, uint8_t *syn,
                            hipStream_t stream) {
    syndrome_kernel<<<dim3(tiles(c.Z), c.mb, F), dim3(kBlock), 0, stream>>>(c, bits, syn);
    return hipGetLastError();
}

}  // namespace ldpc
