// Device-side building blocks of the decoder: Phi, the check update, the
// variable update, and the per-decode set-up and read-out steps, each for one
// (frame, row or column, tile) work item.  Shared by the single-call decoder
// (decoder.hip) and the multi-request engine (engine.hip), so both run the
// same arithmetic in the same order.
#pragma once

#include "internal.h"

#include <hip/hip_fp16.h>

namespace ldpc {
namespace dev {

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
    int vote;                  // 1: record the check of iteration t-1 (t when vote-only)
    int d1_from_llr;           // vote-only at t = 0: decisions come from the channel signs
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

// Checks per thread (CPT): a thread handles checks a, a + 256, ..., a + 256 (CPT-1)
// of one row, so the row's table reads are paid once and every thread has its
// loads for several checks in flight together.  A row's Z checks take
// ceil(Z / (256 CPT)) workgroups, i.e. 4 ceil(Z / (256 CPT)) wavefronts per
// circulant block: the schedule knob the autotuner sets (1, 2 or 4).
inline unsigned check_tiles(int Z, int cpt) {
    return (unsigned)((Z + kBlock * cpt - 1) / (kBlock * cpt));
}
// how many of those are processed at once (bounded by registers for large D)
template <int D> struct ChunkOf { static constexpr int value = D <= 4 ? 2 : 1; };

// What a check-pass launch does; a template parameter, so that each launch is
// straight-line code that issues all of a chunk's loads before it waits.
enum : int {
    kSteady = 0,    // iteration t >= 2: read the old messages, vote t-1 from stored bits
    kFirst = 1,     // iteration 1: old messages are zero, vote t = 0 from the channel signs
    kVoteOnly = 2,  // no update: only the parity check of the last iteration
};

// K checks (r, a_first + q*256), q < K, of one frame, row degree D with DS
// stored blocks.  Padding lanes (a >= Z) load from a clamped in-range index,
// take part in the wave ballots with zero bits and store nothing.  Returns 1
// if one of this thread's checks fails the parity check of the voted iteration.
template <int D, int DS, int K, int MODE, typename Msg>
__device__ __forceinline__ int check_chunk(const RowCtx<D, Msg> &R, const CnArgs &A,
                                           unsigned a_first) {
    const unsigned Z = R.Z;
    float x[K][D];  // inputs L_vc of iteration t-1 (degree-1: Psi)
    int vpar[K];    // parity of the voted decisions on each check, with s_c
    int sb[K];      // syndrome bits
#pragma unroll
    for (int q = 0; q < K; ++q) {
        const unsigned a = a_first + q * kBlock;
        const bool valid = a < Z;
        const unsigned al = valid ? a : Z - 1;  // in-range load index
        const unsigned w = al >> 6, bit = al & 63u;
        sb[q] = (int)((at(R.syn, w) >> bit) & 1ull);
        int par = 0;
#pragma unroll
        for (int k = 0; k < D; ++k) {
            unsigned j = al + R.shift[k];
            j -= (j >= Z) ? Z : 0u;
            float xv;
            int dec;
            if (stored<DS>(R, k)) {
                const float lt = at(R.tot, R.src[k] + j);
                dec = lt < 0.0f;
                const float mo = (MODE == kSteady) ? msg_load<Msg>(&at(R.msg, R.off[k] + al)) : 0.0f;
                xv = lt - mo;
            } else {
                xv = at(R.psi, R.off[k] + al);
                if (MODE == kFirst) {
                    dec = xv < 0.0f;
                } else {
                    const int db = (int)((at(R.d1_prev, R.wrd[k] + w) >> bit) & 1ull);
                    dec = (MODE == kVoteOnly && A.d1_from_llr) ? (xv < 0.0f) : db;
                }
            }
            x[q][k] = xv;
            par ^= dec;
        }
        vpar[q] = valid ? (par ^ sb[q]) : 0;
    }
    int bad = 0;
#pragma unroll
    for (int q = 0; q < K; ++q) bad |= vpar[q];
    if (MODE == kVoteOnly) return bad;

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

template <int D, int DS, int MODE, typename Msg, int CPT>
__device__ __forceinline__ void check_row(const CodeDev &c, const CnArgs &A, int f, int r,
                                          unsigned tile) {
    const RowCtx<D, Msg> R = load_row<D, Msg>(c, A, f, r);
    constexpr int K = ChunkOf<D>::value < CPT ? ChunkOf<D>::value : CPT;
    const unsigned a0 = tile * (kBlock * CPT) + threadIdx.x;
    int bad = 0;
#pragma unroll
    for (int q0 = 0; q0 < CPT; q0 += K)
        bad |= check_chunk<D, DS, K, MODE, Msg>(R, A, a0 + q0 * kBlock);
    if (A.vote) {
        // One flag per frame and iteration, set by any workgroup holding an
        // unsatisfied check.  Every writer stores the same value, so plain
        // stores suffice; reading first keeps all but a few workgroups per
        // frame from storing at all (the next launch sees the stores).
        bad = __syncthreads_or(bad);
        if (bad && threadIdx.x == 0) {
            int32_t *flag = A.fail + (size_t)(MODE == kVoteOnly ? A.t : A.t - 1) * A.F + f;
            if (*reinterpret_cast<volatile int32_t *>(flag) == 0) *flag = 1;
        }
    }
}

// Check update of one (frame, row, tile) work item: dispatch on the row's
// degree and number of stored blocks.  The common rows (degree <= 6 with at
// most one degree-1 block, as in multi-edge codes) are compiled for every
// (degree, stored blocks) pair; every other row goes to the generic class,
// compiled per degree with the split read at run time.
template <typename Msg, bool kLarge, int MODE, int CPT>
__device__ __forceinline__ void check_work(const CodeDev &c, const CnArgs &A, int f, int r,
                                           unsigned tile) {
#define LDPC_CASE(D) \
    case D: check_row<D, -1, MODE, Msg, CPT>(c, A, f, r, tile); break;
#define LDPC_CASE2(D, S) \
    case (D) * 32 + (S): check_row<D, S, MODE, Msg, CPT>(c, A, f, r, tile); break;
    if (!kLarge) {
        static_assert(kSmallRowDegree == 6, "case list below covers degrees 1..6");
        switch (c.row_deg[r] * 32 + c.row_ns[r]) {
            LDPC_CASE2(1, 0) LDPC_CASE2(1, 1) LDPC_CASE2(2, 1) LDPC_CASE2(2, 2)
            LDPC_CASE2(3, 2) LDPC_CASE2(3, 3) LDPC_CASE2(4, 3) LDPC_CASE2(4, 4)
            LDPC_CASE2(5, 4) LDPC_CASE2(5, 5) LDPC_CASE2(6, 5) LDPC_CASE2(6, 6)
            default: break;
        }
    } else {
        static_assert(LDPC_MAX_ROW_DEGREE == 16, "case list below covers degrees 1..16");
        switch (c.row_deg[r]) {
            LDPC_CASE(1) LDPC_CASE(2) LDPC_CASE(3) LDPC_CASE(4) LDPC_CASE(5) LDPC_CASE(6)
            LDPC_CASE(7) LDPC_CASE(8) LDPC_CASE(9) LDPC_CASE(10) LDPC_CASE(11) LDPC_CASE(12)
            LDPC_CASE(13) LDPC_CASE(14) LDPC_CASE(15) LDPC_CASE(16)
            default: break;
        }
    }
#undef LDPC_CASE
#undef LDPC_CASE2
}

struct VnArgs {
    const float *llr;
    const void *msg;
    float *tot;
    const int32_t *fail;
    size_t msg_frame, tot_frame;
    int F, t;
};

// Loads per batch of the variable pass for columns of degree <= max_deg: about
// 20 per batch, rounded up to an instantiated width (8, 11, 16, 17, 21, 26).
inline int variable_batch(int max_deg) {
    const int nb = max_deg <= 0 ? 1 : (max_deg + 19) / 20;
    const int u = (max_deg + nb - 1) / nb;
    for (int w : {8, 11, 16, 17, 21, 26})
        if (u <= w) return w;
    return 26;
}

// Step 3 for the core columns: L_v = Q_v + sum of the column's messages, in
// increasing row order.  One thread per (core column k, position j).  The
// messages are loaded U at a time with all U loads in flight together (a
// column of degree <= U takes one batch); slots past the column's degree load
// a clamped in-range entry and add 0.
template <int U, typename Msg>
__device__ __forceinline__ void variable_work(const CodeDev &c, const VnArgs &A, int f, int k,
                                              unsigned tile) {
    const unsigned Z = (unsigned)c.Z;
    const unsigned j = tile * kBlock + threadIdx.x;
    if (j >= Z) return;
    const Msg *msg = reinterpret_cast<const Msg *>(A.msg) + (size_t)f * A.msg_frame;
    const float *llr = A.llr + (size_t)f * c.n + (size_t)c.core_col[k] * Z;
    float L = at(llr, j);
    const int i0 = c.core_first[k], deg = c.core_deg[k];
    for (int b = 0; b < deg; b += U) {
        float v[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int i = i0 + min(b + u, deg - 1);
            const unsigned s = (unsigned)c.core_shift[i];
            const unsigned idx = (j >= s) ? j - s : j + Z - s;
            v[u] = msg_load<Msg>(&at(msg, (unsigned)c.core_state[i] * Z + idx));
        }
#pragma unroll
        for (int u = 0; u < U; ++u) L += (b + u < deg) ? v[u] : 0.0f;
    }
    at(A.tot + (size_t)f * A.tot_frame, (unsigned)k * Z + j) = L;
}

// Pack the syndrome bytes into 64-bit words per base row: bit a%64 of word a/64.
__device__ __forceinline__ void pack_syndrome_work(const CodeDev &c, const uint8_t *syn,
                                                   uint64_t *synbits, size_t syn_frame, int f, int r,
                                                   unsigned tile) {
    const int a = tile * kBlock + threadIdx.x;
    const bool valid = a < c.Z;
    const int v = valid ? (syn[(size_t)f * c.m + (size_t)r * c.Z + a] & 1) : 0;
    const unsigned long long bits = wave_ballot(v != 0);
    if ((threadIdx.x & 63) == 0 && valid)
        synbits[(size_t)f * syn_frame + (size_t)r * c.W + (a >> 6)] = bits;
}

// Core totals of iteration 0: L_v = Q_v.
__device__ __forceinline__ void init_totals_work(const CodeDev &c, const float *llr, float *tot,
                                                 size_t tot_frame, int f, int k, unsigned tile) {
    const int j = tile * kBlock + threadIdx.x;
    if (j >= c.Z) return;
    tot[(size_t)f * tot_frame + (size_t)k * c.Z + j] =
        llr[(size_t)f * c.n + (size_t)c.core_col[k] * c.Z + j];
}

// Degree-1 inputs in check order: Psi[a] = +-Phi(|Q_p|), p the variable of
// check a of degree-1 block k, with the sign of Q_p (negative iff Q_p < 0).
__device__ __forceinline__ void init_psi_work(const CodeDev &c, const float *llr, float *psi,
                                              size_t psi_frame, int f, int k, unsigned tile) {
    const unsigned Z = (unsigned)c.Z;
    const unsigned a = tile * kBlock + threadIdx.x;
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

// Exit iteration and converged flag of frame f: the first checked iteration
// whose parity check succeeded (fail flag 0), else max_iters and 0.  One
// wave64 per frame scans 64 iterations per step with a ballot.
__device__ __forceinline__ void frame_exit_work(const FinArgs &A, int f) {
    const int lane = threadIdx.x & 63;
    int it = A.T, conv = 0;
    for (int t0 = 0; t0 <= A.T; t0 += 64) {
        const int t = t0 + lane;
        const bool ok = t <= A.T && A.fail[(size_t)t * A.F + f] == 0;
        const unsigned long long m = wave_ballot(ok);
        if (m) {
            it = t0 + __builtin_ctzll(m);
            conv = 1;
            break;
        }
    }
    if (lane == 0) {
        A.iters_out[f] = it;
        A.conv_out[f] = (uint8_t)conv;
    }
}

// Read-out of frame f (after frame_exit_work): hard decisions and posteriors at
// the exit iteration.
__device__ __forceinline__ void finalize_work(const CodeDev &c, const FinArgs &A, int f,
                                              unsigned tile) {
    const int it = A.iters_out[f];
    const int v = tile * kBlock + threadIdx.x;
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


}  // namespace dev
}  // namespace ldpc
