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

// Work items of a launch in XCD-aware order.  The hardware hands consecutive
// workgroups to the chip's 8 XCDs in turn, and each XCD has its own L2.
// Workgroup g takes item (g mod 8) * per + g / 8, so XCD x runs the
// contiguous items [x per, (x + 1) per): items that share data (one frame's
// core totals, the lines at the edges of neighbouring tiles) meet in one L2.
constexpr unsigned kXcds = 8;
inline unsigned xcd_grid(unsigned n) { return (n + kXcds - 1) / kXcds * kXcds; }
__device__ __forceinline__ unsigned xcd_item(unsigned g, unsigned n) {
    const unsigned per = (n + kXcds - 1) / kXcds;
    return (g % kXcds) * per + g / kXcds;
}
// Division by a launch constant d with a multiplier the host computes: for
// every x < 2^31, floor(x / d) = (x m) >> l with l = 31 + ceil(log2 d) and
// m = ceil(2^l / d) (the rounding error x (m d - 2^l) / (d 2^l) stays below
// 2^-ceil(log2 d) <= 1/d).
struct FastDiv {
    uint32_t d, m, l;
};
inline FastDiv fast_div(uint32_t d) {
    uint32_t c = 0;
    while ((1ull << c) < d) ++c;
    const uint32_t l = 31 + c;
    return FastDiv{d, (uint32_t)(((1ull << l) + d - 1) / d), l};
}
__device__ __forceinline__ uint32_t fdiv(uint32_t x, const FastDiv &f) {
    return (uint32_t)(((uint64_t)x * f.m) >> f.l);
}

// Units.  On the device every log-likelihood ratio of the decoding state
// (core totals, messages, degree-1 inputs) is held in base 2: b = L log2(e),
// the natural-log value L scaled by 1/ln 2.  Channel LLRs come in and
// posteriors go out in natural units.  In base 2 the exponential inside Phi is
// a bare exp2 and Phi keeps its involution form, so one function serves
// both directions of the check update.
constexpr float kLog2e = 1.4426950408889634f;
constexpr float kLn2 = 0.6931471805599453f;
// The clamp [1e-7, 30] of Phi's argument, in base-2 units.
constexpr float kPhiLo = 1.442695066e-07f;
constexpr float kPhiHi = 4.328084946e+01f;

// Phi in base-2 units: phi2(b) = log2(e) Phi(b ln 2), where Phi(x) =
// -ln tanh(x/2); like Phi it is a decreasing involution.  Argument clamped to
// [kPhiLo, kPhiHi] (the natural-unit clamp [1e-7, 30]).  Branch-free:
//   b <  1.5 log2(e): phi2(b) = 1 - log2(ln 2) - log2(b) + w H(w), w = b^2,
//                     H a degree-3 near-minimax fit of the smooth remainder
//                     (the expansion of -ln(tanh(y)/y) about 0, rescaled);
//   b >= 1.5 log2(e): phi2(b) = log2(e) 2 atanh(t), t = 2^-b = e^-x, by its
//                     odd series to t^7 (t <= 0.223; truncation below 7e-7).
// Each branch takes one hardware transcendental (log2 or exp2).  Relative
// error in FP32 below 1e-6 over the whole clamped range.
struct PhiConsts {
    float h3, h2, h1, h0, a, p3, p2, p1, p0, hi;  // polynomial coefficients, clamp bound
};

__device__ __forceinline__ float opaque(float v) {
    asm volatile("" : "+v"(v));
    return v;
}

// The constants an FMA cannot take as its one literal, held in registers for
// a whole launch: each passes through an empty asm statement once, so the
// compiler keeps it instead of re-materialising it before every use.
__device__ __forceinline__ PhiConsts phi_consts() {
    PhiConsts K;
    K.h3 = opaque(-1.304959028e-06f);
    K.h2 = opaque(5.194569894e-05f);
    K.h1 = opaque(-1.614399021e-03f);
    K.h0 = opaque(5.775980651e-02f);
    K.a = opaque(1.528766394e+00f);
    K.p3 = opaque(4.121985734e-01f);
    K.p2 = opaque(5.770780444e-01f);
    K.p1 = opaque(9.617967010e-01f);
    K.p0 = opaque(2.885390043e+00f);
    K.hi = opaque(kPhiHi);
    return K;
}

__device__ __forceinline__ float phi2(float b, const PhiConsts &K) {
    b = __builtin_amdgcn_fmed3f(b, kPhiLo, K.hi);
    const float w = b * b;
    float h = fmaf(w, K.h3, K.h2);
    h = fmaf(h, w, K.h1);
    h = fmaf(h, w, K.h0);
    const float small = fmaf(h, w, K.a) - __builtin_amdgcn_logf(b);
    const float t = __builtin_amdgcn_exp2f(-b);
    const float t2 = t * t;
    float p = fmaf(t2, K.p3, K.p2);
    p = fmaf(t2, p, K.p1);
    p = fmaf(t2, p, K.p0);
    const float large = t * p;
    return b < 2.164042473e+00f ? small : large;
}

__device__ __forceinline__ float phi2(float b) { return phi2(b, phi_consts()); }

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
// The value a message reads back as after msg_store.
template <typename Msg> __device__ __forceinline__ float msg_round(float v);
template <> __device__ __forceinline__ float msg_round<float>(float v) { return v; }
template <> __device__ __forceinline__ float msg_round<_Float16>(float v) {
    return static_cast<float>(static_cast<_Float16>(v));
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
    float *part;               // [F][n_groups][Zp] owner-group partial sums (grouped launches)
    size_t msg_frame, tot_frame, d1_frame, syn_frame, psi_frame, part_frame;
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
    unsigned off[D];          // state: msg offset ref*Zp; degree-1: psi offset ref*Zp
    unsigned src[D];          // state: totals offset core*Zt; degree-1: llr offset col*Z
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
        R.off[k] = ref * (unsigned)c.Zp;
        R.src[k] = st ? (unsigned)c.blk_core[b] * (unsigned)c.Zt : (unsigned)c.blk_col[b] * Z;
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
    kPost = 4,      // flag on kSteady / kFirst: also write degree-1 posteriors Q + m
};
constexpr int base_mode(int mode) { return mode & 3; }
constexpr bool with_post(int mode) { return (mode & kPost) != 0; }

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
                const float mo = (base_mode(MODE) == kSteady) ? msg_load<Msg>(&at(R.msg, R.off[k] + al)) : 0.0f;
                xv = lt - mo;
            } else {
                xv = at(R.psi, R.off[k] + al);
                if (base_mode(MODE) == kFirst) {
                    dec = xv < 0.0f;
                } else {
                    const int db = (int)((at(R.d1_prev, R.wrd[k] + w) >> bit) & 1ull);
                    dec = (base_mode(MODE) == kVoteOnly && A.d1_from_llr) ? (xv < 0.0f) : db;
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
    if (base_mode(MODE) == kVoteOnly) return bad;

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
            ph[k] = stored<DS>(R, k) ? phi2(fabsf(x[q][k])) : fabsf(x[q][k]);
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
                const float mag = phi2(ex[k]);
                if (valid) msg_store<Msg>(&at(R.msg, R.off[k] + a), sgn ? -mag : mag);
            } else {
                // decision of the degree-1 variable: sign of Q + m
                const int negq = (neg >> k) & 1;
                const float S = __builtin_amdgcn_fmed3f(ex[k], kPhiLo, kPhiHi);
                const int dec = (negq == sgn) ? negq : (ph[k] < S ? negq : sgn);
                const unsigned long long bits = wave_ballot(valid && dec);
                if ((threadIdx.x & 63) == 0 && valid) at(R.d1_cur, R.wrd[k] + w) = bits;
                if (with_post(MODE) && R.d1post && valid) {
                    unsigned j = a + R.shift[k];
                    j -= (j >= Z) ? Z : 0u;
                    const float mag = phi2(ex[k]) * kLn2;
                    at(R.d1post, R.off[k] + a) = at(R.llr, R.src[k] + j) + (sgn ? -mag : mag);
                }
            }
        }
    }
    return bad;
}

// Bit l of a wave-uniform 64-bit word as lane l's predicate: the word is used
// directly as a lane mask, with no per-lane shift.
__device__ __forceinline__ bool lane_bit(uint64_t word) {
    return __builtin_amdgcn_inverse_ballot_w64(word);
}

// A 64-bit word at a wave-uniform address that no lane of the running launch
// writes (syndrome bits, decision bits of the previous iteration): read with a
// scalar load.
__device__ __forceinline__ uint64_t uniform_word(const uint64_t *p) {
    typedef const __attribute__((address_space(4))) uint64_t ConstWord;
    return *(ConstWord *)p;
}

// A 32-bit value at a wave-uniform address, read with a scalar load.  Used
// for tables and flags that this launch does not write, and for the vote flag,
// where a stale 0 only costs one redundant store of the same value.
__device__ __forceinline__ int32_t uniform_i32(const int32_t *p) {
    typedef const __attribute__((address_space(4))) int32_t ConstI32;
    return *(ConstI32 *)p;
}

// Workgroup-uniform pointers of one (frame, row) for rows whose split into
// DS stored blocks followed by D - DS degree-1 blocks is a compile-time fact.
// A thread's checks are a0 + 256 q; the wave's 64 checks of step q are bit
// positions 0..63 of word w0 + 4 q of every packed bit array of the row, so
// syndrome and decision bits are whole uniform words, one bit per lane.
template <int D, int DS, typename Msg>
struct FixedRow {
    const float *tot[D];        // stored k: totals row of the block's column, advanced by its shift
    Msg *msg[D];                // stored k: the block's messages
    const float *psi[D];        // degree-1 k: Psi of the block's variables, check order
    const uint64_t *dprev[D];   // degree-1 k: decision words of iteration t-1
    uint64_t *dcur[D];          // degree-1 k: decision words of iteration t
    const float *llr[D];        // degree-1 k: channel LLRs of the block's column (posteriors only)
    float *post[D];             // degree-1 k: posteriors of iteration t, or null
    unsigned shift[D];
    const uint64_t *syn;        // the row's packed syndrome words
    unsigned Z, Wm1;
    int32_t any_desc;           // OR of the descriptor words read (never negative)
};

// The row at row_list position y, from its descriptor: one burst of scalar
// loads, independent of every other table.
template <int D, int DS, typename Msg>
__device__ __forceinline__ FixedRow<D, DS, Msg> fixed_row(const CodeDev &c, const CnArgs &A, int f,
                                                          int y) {
    FixedRow<D, DS, Msg> R;
    const unsigned Z = (unsigned)c.Z;
    R.Z = Z;
    R.Wm1 = (unsigned)c.W - 1;
    typedef const __attribute__((address_space(4))) int32_t ConstI32;
    ConstI32 *d = (ConstI32 *)(c.row_desc + (size_t)y * kRowDescWords);
    const float *tot = A.tot + (size_t)f * A.tot_frame;
    Msg *msg = reinterpret_cast<Msg *>(A.msg) + (size_t)f * A.msg_frame;
    R.syn = A.synbits + (size_t)f * A.syn_frame + (unsigned)d[16];
    R.any_desc = d[16];
#pragma unroll
    for (int k = 0; k < D; ++k) {
        if (k < DS) {
            R.tot[k] = tot + (unsigned)d[k];
            R.msg[k] = msg + (unsigned)d[6 + k];
            R.any_desc |= d[k] | d[6 + k];
        } else {
            R.any_desc |= d[12] | d[13] | d[14] | d[15];
            R.psi[k] = A.psi + (size_t)f * A.psi_frame + (unsigned)d[12];
            R.dprev[k] = A.d1_prev + (size_t)f * A.d1_frame + (unsigned)d[13];
            R.dcur[k] = A.d1_cur ? A.d1_cur + (size_t)f * A.d1_frame + (unsigned)d[13] : nullptr;
            R.llr[k] = A.llr + (size_t)f * c.n + (unsigned)d[14];
            R.shift[k] = (unsigned)d[15];
            R.post[k] = A.d1post ? A.d1post + (size_t)f * A.psi_frame + (unsigned)d[12] : nullptr;
        }
    }
    return R;
}

// Step 2 of one check of degree D whose first DS inputs are stored edges and
// the others degree-1 inputs (Psi, already in the Phi domain).  From the
// inputs x (L_vc, or Psi): the input signs neg, the Phi values ph and the
// exclusive Phi sums ex, as prefix sums from the left plus suffix sums from
// the right (a fixed order).  Returns the check's sign parity, the syndrome
// bit included: the message to input k is negative iff parity ^ neg[k].
template <int D, int DS>
__device__ __forceinline__ bool phi_exclusive(const float (&x)[D], bool syn, const PhiConsts &PK,
                                              bool (&neg)[D], float (&ph)[D], float (&ex)[D]) {
    bool par = syn;
#pragma unroll
    for (int k = 0; k < D; ++k) {
        neg[k] = x[k] < 0.0f;
        par ^= neg[k];
        ph[k] = (k < DS) ? phi2(fabsf(x[k]), PK) : fabsf(x[k]);
    }
    if constexpr (D == 1) {
        ex[0] = 0.0f;
    } else {
        float pre[D];
        pre[0] = 0.0f;
#pragma unroll
        for (int k = 1; k < D; ++k) pre[k] = (k == 1) ? ph[0] : pre[k - 1] + ph[k - 1];
        float suf = ph[D - 1];
        ex[D - 1] = pre[D - 1];
#pragma unroll
        for (int k = D - 2; k >= 0; --k) {
            ex[k] = (k == 0) ? suf : pre[k] + suf;
            suf += ph[k];
        }
    }
    return par;
}

// The check update in the t-domain, for a check of degree 3 with two stored
// inputs x1, x2 and one degree-1 input whose channel LLR Q enters as
// tq = e^{-|Q|} (the multi-edge template's type-2 checks, which carry almost
// all checks).  With t = e^{-|x|} (in base-2 units 2^{-b}) the tanh rule
// tanh(m/2) = prod tanh(x_k/2) becomes, for two inputs,
//   t_out = (t_a + t_b) / (1 + t_a t_b),   |m| = -ln t_out,
// which is Phi(Phi(a) + Phi(b)) written out (tanh(x/2) = (1 - t)/(1 + t)).
// Every term is positive, so nothing cancels, and each message costs one
// reciprocal and one logarithm instead of two Phi evaluations.  The clamps
// of the Phi arguments carry over exactly: the forward clamp of |x| to
// [1e-7, 30] clamps b before the exponential, and the clamp of the inverse
// argument (the exclusive Phi sum) to [1e-7, 30] is, Phi being decreasing,
// a clamp of |m| to [Phi(30), Phi(1e-7)].  Accuracy: |m| within 3.2e-7 *
// max(|m|, 1) of the double-precision definition over inputs 1e-9 .. 40.
// Outputs (base 2): |m| to input 1 (from x2 and Q), |m| to input 2 (from x1
// and Q), and whether the degree-1 variable's |Q| exceeds the clamped |m|
// of the message from x1 and x2 (its decision then follows Q).
constexpr float kMsgLo = 2.7000394e-13f;  // Phi(30) log2(e)
constexpr float kMsgHi = 2.4253496e+01f;  // Phi(1e-7) log2(e)
constexpr float kTLo = 5.0000020e-08f;    // 2^-kMsgHi = e^{-Phi(1e-7)}

__device__ __forceinline__ float tdom_mag(float ta, float tb) {
    const float num = fmaf(ta, tb, 1.0f);
    const float r = num * __builtin_amdgcn_rcpf(ta + tb);
    return __builtin_amdgcn_fmed3f(__builtin_amdgcn_logf(r), kMsgLo, kMsgHi);
}

__device__ __forceinline__ void tdom_check3(float x1, float x2, float tq, const PhiConsts &PK,
                                            float &mag1, float &mag2, bool &q_wins, float &t1o,
                                            float &t2o) {
    const float t1 = __builtin_amdgcn_exp2f(-__builtin_amdgcn_fmed3f(fabsf(x1), kPhiLo, PK.hi));
    const float t2 = __builtin_amdgcn_exp2f(-__builtin_amdgcn_fmed3f(fabsf(x2), kPhiLo, PK.hi));
    mag1 = tdom_mag(tq, t2);
    mag2 = tdom_mag(tq, t1);
    // |Q| > min(|m_p|, Phi(1e-7)): tq < max(t_p, kTLo), t_p = (t1 + t2) / (1 + t1 t2)
    q_wins = (tq < kTLo) | (tq * fmaf(t1, t2, 1.0f) < t1 + t2);
    t1o = t1;
    t2o = t2;
}

// The degree-1 input a check reads for variable p: its channel LLR Q_p in the
// form the check's update takes, with the sign of Q_p: +-Phi(|Q_p|) for the
// Phi-domain update, +-e^{-|Q_p|} for the t-domain one (base 2 throughout;
// |Q| clamped to [1e-7, 30] either way).
__device__ __forceinline__ float d1_input(float q, bool tdom, const PhiConsts &PK) {
    const float b = fabsf(q) * kLog2e;
    const float p = tdom ? __builtin_amdgcn_exp2f(-__builtin_amdgcn_fmed3f(b, kPhiLo, PK.hi))
                         : phi2(b, PK);
    return q < 0.0f ? -p : p;
}

// Decision of a degree-1 variable: the sign of Q + m, taken in the Phi domain
// (|Q| > |m| exactly when Phi(|Q|) < S, S the exclusive sum of the check's
// other inputs).  The signs of Q and m differ exactly when the check's whole
// sign parity is odd; then the larger magnitude decides.
__device__ __forceinline__ bool d1_decision(bool neg, bool par, float ph, float ex,
                                            const PhiConsts &PK) {
    const float S = __builtin_amdgcn_fmed3f(ex, kPhiLo, PK.hi);
    return neg ^ (par && !(ph < S));
}

// K checks a + 256 q (q < K) of a fixed row; w = the wave's word of check a.
// Padding lanes (check >= Z) read in-bounds slack (the row stride of the
// totals and the padding after the message and Psi regions cover them), are
// masked out of the vote and the decision words, and store nothing.  Returns
// true if one of this thread's checks fails the parity check of the voted
// iteration.
template <int D, int DS, int K, int MODE, typename Msg>
__device__ __forceinline__ bool fixed_chunk(const FixedRow<D, DS, Msg> &R, const CnArgs &A,
                                            unsigned a, unsigned w, const PhiConsts &PK) {
    float lt[K][D];  // stored k: totals of iteration t-1; degree-1 k: Psi
    float mo[K][D];  // stored k: messages of iteration t-1
    uint64_t sw[K];  // syndrome words
    uint64_t dw[K][D];  // degree-1 k: decision words of iteration t-1
#pragma unroll
    for (int q = 0; q < K; ++q) {
        const unsigned wq = min(w + 4u * q, R.Wm1);
        sw[q] = uniform_word(R.syn + wq);
#pragma unroll
        for (int k = 0; k < D; ++k) {
            if (k < DS) {
                lt[q][k] = at(R.tot[k] + q * kBlock, a);
                mo[q][k] = (base_mode(MODE) == kSteady) ? msg_load<Msg>(&at(R.msg[k] + q * kBlock, a))
                                                        : 0.0f;
            } else {
                lt[q][k] = at(R.psi[k] + q * kBlock, a);
                if (base_mode(MODE) != kFirst) dw[q][k] = uniform_word(R.dprev[k] + wq);
            }
        }
    }
    float x[K][D];  // inputs L_vc of iteration t-1 (degree-1: Psi)
    bool dec[K][D]; // decisions of the voted iteration
#pragma unroll
    for (int q = 0; q < K; ++q) {
#pragma unroll
        for (int k = 0; k < D; ++k) {
            if (k < DS) {
                x[q][k] = lt[q][k] - mo[q][k];
                dec[q][k] = lt[q][k] < 0.0f;
            } else {
                x[q][k] = lt[q][k];
                if (base_mode(MODE) == kFirst)
                    dec[q][k] = x[q][k] < 0.0f;
                else if (base_mode(MODE) == kVoteOnly && A.d1_from_llr)
                    dec[q][k] = x[q][k] < 0.0f;
                else
                    dec[q][k] = lane_bit(dw[q][k]);
            }
        }
    }
    bool bad = false;
#pragma unroll
    for (int q = 0; q < K; ++q) {
        bool par = lane_bit(sw[q]);
#pragma unroll
        for (int k = 0; k < D; ++k) par ^= dec[q][k];
        bad |= par && (a + q * kBlock < R.Z);
    }
    if (base_mode(MODE) == kVoteOnly) return bad;

#pragma unroll
    for (int q = 0; q < K; ++q) {
        const unsigned aq = a + q * kBlock;
        const bool valid = aq < R.Z;
        // Step 2: sign product with the syndrome bit, Phi-domain exclusive sums
        float ph[D], ex[D];
        bool neg[D];
        const bool par = phi_exclusive<D, DS>(x[q], lane_bit(sw[q]), PK, neg, ph, ex);
#pragma unroll
        for (int k = 0; k < D; ++k) {
            const bool sgn = par ^ neg[k];  // the message to block k is negative
            if (k < DS) {
                const float mag = phi2(ex[k], PK);
                if (valid) msg_store<Msg>(&at(R.msg[k] + q * kBlock, a), sgn ? -mag : mag);
            } else {
                const bool d = d1_decision(neg[k], par, ph[k], ex[k], PK);
                const unsigned long long bits = wave_ballot(valid && d);
                if ((threadIdx.x & 63) == 0 && valid) at(R.dcur[k], w + 4u * q) = bits;
                if constexpr (with_post(MODE)) {
                    if (valid) {
                        unsigned j = aq + R.shift[k];
                        j -= (j >= R.Z) ? R.Z : 0u;
                        const float mag = phi2(ex[k], PK) * kLn2;
                        at(R.post[k], aq) = at(R.llr[k], j) + (sgn ? -mag : mag);
                    }
                }
            }
        }
    }
    return bad;
}

// Sign bit of v as the decisions and sign products read it: set iff v < 0
// (-0 adds to +0, so it counts as non-negative, as L >= 0 decides 0).
constexpr uint32_t kSignBit = 0x80000000u;
__device__ __forceinline__ uint32_t neg_bit(float v) {
    return __float_as_uint(v + 0.0f) & kSignBit;
}

// A row of class (degree 3, 2 stored blocks, 1 degree-1 block): the
// template's type-2 checks, almost all checks of a multi-edge code.  Wave
// `wave` of tile `tile` takes CPT consecutive chunks of 64 checks, check
// a = tile 256 CPT + wave 64 CPT + 64 q + lane for chunk q, so its packed bit
// words (syndrome, previous and new degree-1 decisions) are CPT consecutive
// words: one scalar load each, one store of the new ones.  Step 2 runs in the
// t-domain (tdom_check3), and the sign products, the parity vote of the
// previous iteration and the degree-1 decision are formed on sign bits in
// vector registers.  FULL: every check of the tile is in the row (a < Z);
// else padding lanes read in-bounds slack (as fixed_chunk), vote nothing and
// store nothing.  The packed-word loads may read up to CPT - 1 words past a
// row's last word; the decode workspace places other regions after every bit
// array, so those reads stay inside it.  Returns true if one of this
// thread's checks fails the parity check of the voted iteration.
template <int MODE, typename Msg, int CPT, bool FULL>
__device__ __forceinline__ bool tdom_chunks(const FixedRow<3, 2, Msg> &R, const CnArgs &A,
                                            unsigned tile, unsigned wave, const PhiConsts &PK) {
    const unsigned lane = threadIdx.x & 63u;
    const unsigned a0 = tile * (kBlock * CPT) + wave * (64u * CPT) + lane;
    const unsigned w0 = tile * (4u * CPT) + wave * CPT;
    struct Words { uint64_t w[CPT]; };
    Words sw, dw{};
#pragma unroll
    for (int q = 0; q < CPT; ++q) {
        sw.w[q] = uniform_word(R.syn + w0 + q);
        if constexpr (base_mode(MODE) != kFirst) dw.w[q] = uniform_word(R.dprev[2] + w0 + q);
    }
    float lt[CPT][2], mo[CPT][2], ps[CPT];
#pragma unroll
    for (int q = 0; q < CPT; ++q) {
        const unsigned a = a0 + 64u * q;
#pragma unroll
        for (int k = 0; k < 2; ++k) {
            lt[q][k] = at(R.tot[k], a);
            mo[q][k] = (base_mode(MODE) == kSteady) ? msg_load<Msg>(&at(R.msg[k], a)) : 0.0f;
        }
        ps[q] = at(R.psi[2], a);
    }
    uint32_t bad = 0;
    uint64_t dbits[CPT];
#pragma unroll
    for (int q = 0; q < CPT; ++q) {
        const unsigned a = a0 + 64u * q;
        const bool valid = FULL || a < R.Z;
        const uint32_t syn = lane_bit(sw.w[q]) ? kSignBit : 0u;
        const uint32_t s2 = __float_as_uint(ps[q]) & kSignBit;  // sign of Q (never -0)
        // parity of the voted decisions: core totals of iteration t-1, and the
        // degree-1 decisions (channel signs at the first iteration)
        uint32_t d1 = s2;
        if constexpr (base_mode(MODE) != kFirst)
            if (!(base_mode(MODE) == kVoteOnly && A.d1_from_llr)) d1 = lane_bit(dw.w[q]) ? kSignBit : 0u;
        const uint32_t vpar = syn ^ neg_bit(lt[q][0]) ^ neg_bit(lt[q][1]) ^ d1;
        bad |= valid ? vpar : 0u;
        if constexpr (base_mode(MODE) == kVoteOnly) continue;
        // Step 2: magnitudes in the t-domain, signs from the exclusive parities
        const float x0 = lt[q][0] - mo[q][0], x1 = lt[q][1] - mo[q][1];
        const uint32_t s0 = neg_bit(x0), s1 = neg_bit(x1);
        float mag0, mag1, t1, t2;
        bool q_wins;
        tdom_check3(x0, x1, fabsf(ps[q]), PK, mag0, mag1, q_wins, t1, t2);
        const float m0 = __uint_as_float(__float_as_uint(mag0) | (syn ^ s1 ^ s2));
        const float m1 = __uint_as_float(__float_as_uint(mag1) | (syn ^ s0 ^ s2));
        if (valid) {
            msg_store<Msg>(&at(R.msg[0], a), m0);
            msg_store<Msg>(&at(R.msg[1], a), m1);
        }
        // degree-1 decision: the sign of Q, unless the check's message to it
        // has the other sign (odd parity) and the larger magnitude
        const uint32_t par = syn ^ s0 ^ s1 ^ s2;
        const uint32_t d = s2 ^ (q_wins ? 0u : par);
        dbits[q] = wave_ballot(valid && d != 0u);
        if constexpr (with_post(MODE)) {
            if (valid) {
                unsigned j = a + R.shift[2];
                j -= (j >= R.Z) ? R.Z : 0u;
                const float mp = tdom_mag(t1, t2) * kLn2;
                at(R.post[2], a) = at(R.llr[2], j) + ((syn ^ s0 ^ s1) ? -mp : mp);
            }
        }
    }
    if constexpr (base_mode(MODE) != kVoteOnly) {
        // lanes 0 .. CPT-1 store the CPT consecutive decision words
        if (lane < (unsigned)CPT) {
            uint64_t v = dbits[0];
#pragma unroll
            for (int q = 1; q < CPT; ++q) v = (lane == (unsigned)q) ? dbits[q] : v;
            if (FULL || w0 + lane <= R.Wm1) at(R.dcur[2], w0 + lane) = v;
        }
    }
    return bad != 0u;
}

// How many of a thread's checks of a fixed row are processed at once (bounded
// by registers for larger rows).
template <int D> struct FixedChunk { static constexpr int value = D <= 3 ? 4 : 1; };

// The flag of the iteration a check-pass launch votes.
template <int MODE>
__device__ __forceinline__ int32_t *vote_flag(const CnArgs &A, int f) {
    return A.fail + (size_t)(base_mode(MODE) == kVoteOnly ? A.t : A.t - 1) * A.F + f;
}

// One flag per frame and iteration, set by any wave holding an unsatisfied
// check.  Every writer stores the same value, so plain stores suffice; waves
// that found the flag already set when their launch began store nothing.
__device__ __forceinline__ void vote_store(int32_t *flag, int32_t seen, bool bad) {
    const bool wave_bad = wave_ballot(bad) != 0ull;
    if (wave_bad && seen == 0 && (threadIdx.x & 63) == 0) *flag = 1;
}

// A common row at row_list position y, (degree, stored blocks) known at
// compile time.  The frame-skip flag, the vote flag and the row descriptor
// are independent scalar loads, issued together before the first wait.
template <int D, int DS, int MODE, typename Msg, int CPT>
__device__ __forceinline__ void check_row_fixed(const CodeDev &c, const CnArgs &A, int f, int y,
                                                unsigned tile) {
    // The flag loads are unconditional (in bounds either way) scalar loads
    // that issue together with the descriptor loads.
    const PhiConsts PK = phi_consts();
    int32_t *flag = vote_flag<MODE>(A, f);
    const int32_t prev = uniform_i32(A.fail + (size_t)max(A.skip_after, 0) * A.F + f);
    const int32_t seen = uniform_i32(flag);
    const FixedRow<D, DS, Msg> R = fixed_row<D, DS, Msg>(c, A, f, y);
    // The frame is skipped when its earlier check succeeded.  The test also
    // reads the descriptor words (never negative), so their scalar loads issue
    // together with the flag loads instead of after the branch.
    const bool skip = (A.skip_after >= 0) & (prev == 0);
    if (skip | (R.any_desc < 0)) return;
    const unsigned wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    bool bad = false;
    if constexpr (D == 3 && DS == 2) {
        if ((tile + 1) * (kBlock * CPT) <= R.Z)
            bad = tdom_chunks<MODE, Msg, CPT, true>(R, A, tile, wave, PK);
        else
            bad = tdom_chunks<MODE, Msg, CPT, false>(R, A, tile, wave, PK);
    } else {
        constexpr int K = FixedChunk<D>::value < CPT ? FixedChunk<D>::value : CPT;
        const unsigned a0 = tile * (kBlock * CPT) + threadIdx.x;
        const unsigned w0 = tile * (4u * CPT) + wave;
#pragma unroll
        for (int q0 = 0; q0 < CPT; q0 += K)
            bad |= fixed_chunk<D, DS, K, MODE, Msg>(R, A, a0 + q0 * kBlock, w0 + 4u * q0, PK);
    }
    if (A.vote) vote_store(flag, seen, bad);
}

// Any other row (base row r), degree D known at compile time.
template <int D, int MODE, typename Msg, int CPT>
__device__ __forceinline__ void check_row_generic(const CodeDev &c, const CnArgs &A, int f, int r,
                                                  unsigned tile) {
    if (A.skip_after >= 0 && A.fail[(size_t)A.skip_after * A.F + f] == 0) return;
    int32_t *flag = vote_flag<MODE>(A, f);
    const int32_t seen = A.vote ? *flag : 1;
    const RowCtx<D, Msg> R = load_row<D, Msg>(c, A, f, r);
    constexpr int K = ChunkOf<D>::value < CPT ? ChunkOf<D>::value : CPT;
    const unsigned a0 = tile * (kBlock * CPT) + threadIdx.x;
    int bad = 0;
#pragma unroll
    for (int q0 = 0; q0 < CPT; q0 += K)
        bad |= check_chunk<D, -1, K, MODE, Msg>(R, A, a0 + q0 * kBlock);
    if (A.vote) vote_store(flag, seen, bad != 0);
}

// Check update of one (frame, row, tile) work item, the row at position y of
// the row list: dispatch on the row's class.  The common rows (degree <= 6
// with at most one degree-1 block, as in multi-edge codes) are compiled for
// every (degree, stored blocks) class, found from y without a memory load;
// every other row goes to the generic class, compiled per degree with the
// split read at run time.
template <typename Msg, bool kLarge, int MODE, int CPT>
__device__ __forceinline__ void check_work(const CodeDev &c, const CnArgs &A, int f, int y,
                                           unsigned tile) {
#define LDPC_CASE(D) \
    case D: check_row_generic<D, MODE, Msg, CPT>(c, A, f, r, tile); break;
#define LDPC_CLASS(I, D, S) \
    case I: check_row_fixed<D, S, MODE, Msg, CPT>(c, A, f, y, tile); break;
    if (!kLarge) {
        static_assert(kFixedClasses == 12, "class list below covers degrees 1..6");
        int cls = 0;
#pragma unroll
        for (int i = 0; i < kFixedClasses - 1; ++i) cls += (y >= c.cls_end[i]) ? 1 : 0;
        switch (cls) {
            LDPC_CLASS(0, 1, 0) LDPC_CLASS(1, 1, 1) LDPC_CLASS(2, 2, 1) LDPC_CLASS(3, 2, 2)
            LDPC_CLASS(4, 3, 2) LDPC_CLASS(5, 3, 3) LDPC_CLASS(6, 4, 3) LDPC_CLASS(7, 4, 4)
            LDPC_CLASS(8, 5, 4) LDPC_CLASS(9, 5, 5) LDPC_CLASS(10, 6, 5) LDPC_CLASS(11, 6, 6)
            default: break;
        }
    } else {
        static_assert(LDPC_MAX_ROW_DEGREE == 16, "case list below covers degrees 1..16");
        const int r = c.row_list[y];
        switch (c.row_deg[r]) {
            LDPC_CASE(1) LDPC_CASE(2) LDPC_CASE(3) LDPC_CASE(4) LDPC_CASE(5) LDPC_CASE(6)
            LDPC_CASE(7) LDPC_CASE(8) LDPC_CASE(9) LDPC_CASE(10) LDPC_CASE(11) LDPC_CASE(12)
            LDPC_CASE(13) LDPC_CASE(14) LDPC_CASE(15) LDPC_CASE(16)
            default: break;
        }
    }
#undef LDPC_CASE
#undef LDPC_CLASS
}

// Common-row check update of one work item whose class is read from word 18
// of the row's descriptor (used where the class boundaries would cost a load
// before the descriptor's: the multi-request engine).
template <typename Msg, int MODE, int CPT>
__device__ __forceinline__ void check_work_by_desc(const CodeDev &c, const CnArgs &A, int f, int y,
                                                   unsigned tile) {
#define LDPC_CLASS(I, D, S) \
    case I: check_row_fixed<D, S, MODE, Msg, CPT>(c, A, f, y, tile); break;
    static_assert(kFixedClasses == 12, "class list below covers degrees 1..6");
    switch (uniform_i32(c.row_desc + (size_t)y * kRowDescWords + 18)) {
        LDPC_CLASS(0, 1, 0) LDPC_CLASS(1, 1, 1) LDPC_CLASS(2, 2, 1) LDPC_CLASS(3, 2, 2)
        LDPC_CLASS(4, 3, 2) LDPC_CLASS(5, 3, 3) LDPC_CLASS(6, 4, 3) LDPC_CLASS(7, 4, 4)
        LDPC_CLASS(8, 5, 4) LDPC_CLASS(9, 5, 5) LDPC_CLASS(10, 6, 5) LDPC_CLASS(11, 6, 6)
        default: break;
    }
#undef LDPC_CLASS
}

// Workgroup-uniform pointers of one (frame, owner group).
template <typename Msg>
struct GroupView {
    const int32_t *desc;   // the group's row descriptors
    const float *tot, *psi, *llr;
    Msg *msg;
    const uint64_t *syn, *dprev;
    uint64_t *dcur;
    float *post;
    unsigned Z, Wm1;
};

// RB rows k0 .. k0 + RB - 1 of an owner group at position p (check p of each
// row, variable p of the owner column, whose total tv is read once for the
// group); w = the wave's word.  The update of each row is that of
// tdom_chunks, term for term; the new message to the owner column is added
// to psum as it will read back from storage.  All loads of the RB rows are
// issued before the first wait.
template <int MODE, typename Msg, int RB, bool FULL>
__device__ __forceinline__ void group_batch(const GroupView<Msg> &G, int k0, float tv, unsigned p,
                                            unsigned w, float &psum, uint32_t &bad,
                                            const PhiConsts &PK) {
    static_assert(base_mode(MODE) != kVoteOnly, "vote-only launches take the row kernel");
    typedef const __attribute__((address_space(4))) int32_t ConstI32;
    ConstI32 *dp = (ConstI32 *)(G.desc + (size_t)k0 * kGroupDescWords);
    const unsigned lane = threadIdx.x & 63u;
    const bool valid = FULL || p < G.Z;
    unsigned d[RB][kGroupDescWords];
#pragma unroll
    for (int i = 0; i < RB; ++i)
#pragma unroll
        for (int j = 0; j < kGroupDescWords; ++j) d[i][j] = (unsigned)dp[i * kGroupDescWords + j];
    uint64_t sw[RB], dw[RB];
    float lt[RB], mo0[RB], mo1[RB], ps[RB];
#pragma unroll
    for (int i = 0; i < RB; ++i) {
        sw[i] = uniform_word(G.syn + d[i][5] + w);
        dw[i] = (base_mode(MODE) != kFirst) ? uniform_word(G.dprev + d[i][4] + w) : 0ull;
        lt[i] = at(G.tot + d[i][2], p);
        mo0[i] = (base_mode(MODE) == kSteady) ? msg_load<Msg>(&at(G.msg + d[i][0], p)) : 0.0f;
        mo1[i] = (base_mode(MODE) == kSteady) ? msg_load<Msg>(&at(G.msg + d[i][1], p)) : 0.0f;
        ps[i] = at(G.psi + d[i][3], p);
    }
    uint64_t dbits[RB];
#pragma unroll
    for (int i = 0; i < RB; ++i) {
        const uint32_t syn = lane_bit(sw[i]) ? kSignBit : 0u;
        const uint32_t s2 = __float_as_uint(ps[i]) & kSignBit;  // sign of Q (never -0)
        const uint32_t d1 = (base_mode(MODE) == kFirst) ? s2 : (lane_bit(dw[i]) ? kSignBit : 0u);
        const uint32_t vpar = syn ^ neg_bit(tv) ^ neg_bit(lt[i]) ^ d1;
        bad |= valid ? vpar : 0u;
        const float x0 = tv - mo0[i], x1 = lt[i] - mo1[i];
        const uint32_t s0 = neg_bit(x0), s1 = neg_bit(x1);
        float mag0, mag1, t1, t2;
        bool q_wins;
        tdom_check3(x0, x1, fabsf(ps[i]), PK, mag0, mag1, q_wins, t1, t2);
        const float m0 = __uint_as_float(__float_as_uint(mag0) | (syn ^ s1 ^ s2));
        const float m1 = __uint_as_float(__float_as_uint(mag1) | (syn ^ s0 ^ s2));
        if (valid) {
            msg_store<Msg>(&at(G.msg + d[i][0], p), m0);
            msg_store<Msg>(&at(G.msg + d[i][1], p), m1);
        }
        psum += msg_round<Msg>(m0);
        const uint32_t par = syn ^ s0 ^ s1 ^ s2;
        const uint32_t dd = s2 ^ (q_wins ? 0u : par);
        dbits[i] = wave_ballot(valid && dd != 0u);
        if constexpr (with_post(MODE)) {
            if (valid) {
                unsigned j = p + d[i][7];
                j -= (j >= G.Z) ? G.Z : 0u;
                const float mp = tdom_mag(t1, t2) * kLn2;
                at(G.post + d[i][3], p) = at(G.llr + d[i][6], j) + ((syn ^ s0 ^ s1) ? -mp : mp);
            }
        }
    }
    // lane i < RB stores row i's decision word
    if (lane < (unsigned)RB) {
        uint64_t v = dbits[0];
        unsigned off = d[0][4];
#pragma unroll
        for (int i = 1; i < RB; ++i) {
            v = (lane == (unsigned)i) ? dbits[i] : v;
            off = (lane == (unsigned)i) ? d[i][4] : off;
        }
        if (FULL || w <= G.Wm1) at(G.dcur + off, w) = v;
    }
}

// Rows of an owner group whose loads are in flight together (measured: 4
// beats 2, 3, 6 and 8 at 24 rows per group, and 3 and 6 at 12).
constexpr int kGroupBatch = 4;

template <int MODE, typename Msg, bool FULL>
__device__ __forceinline__ void group_rows(const GroupView<Msg> &G, int nrows, float tv, unsigned p,
                                           unsigned w, float &psum, uint32_t &bad,
                                           const PhiConsts &PK) {
    int k = 0;
    for (; k + kGroupBatch <= nrows; k += kGroupBatch)
        group_batch<MODE, Msg, kGroupBatch, FULL>(G, k, tv, p, w, psum, bad, PK);
    for (; k < nrows; ++k) group_batch<MODE, Msg, 1, FULL>(G, k, tv, p, w, psum, bad, PK);
}

// Check update of one (frame, owner group g, 256 positions) work item: every
// row of the group at positions p = tile 256 + thread (Alg. 1 Step 2 and the
// Step 4 check of iteration t-1, as for the rows' own work items), plus the
// group's partial sum of the new messages to the owner column, written to
// part[f][g][p].  Padding lanes (p >= Z) read in-bounds slack and store
// nothing, as in tdom_chunks.
template <int MODE, typename Msg>
__device__ __forceinline__ void group_work(const CodeDev &c, const CnArgs &A, int f, int g,
                                           unsigned tile) {
    const PhiConsts PK = phi_consts();
    int32_t *flag = vote_flag<MODE>(A, f);
    const int32_t prev = uniform_i32(A.fail + (size_t)max(A.skip_after, 0) * A.F + f);
    const int32_t seen = uniform_i32(flag);
    const int32_t own = uniform_i32(c.grp_hdr + 4 * g);
    const int32_t nrows = uniform_i32(c.grp_hdr + 4 * g + 1);
    const bool skip = (A.skip_after >= 0) & (prev == 0);
    if (skip | (nrows <= 0)) return;
    GroupView<Msg> G;
    G.desc = c.grp_desc + (size_t)g * kGroupRows * kGroupDescWords;
    G.tot = A.tot + (size_t)f * A.tot_frame;
    G.psi = A.psi + (size_t)f * A.psi_frame;
    G.llr = A.llr + (size_t)f * c.n;
    G.msg = reinterpret_cast<Msg *>(A.msg) + (size_t)f * A.msg_frame;
    G.syn = A.synbits + (size_t)f * A.syn_frame;
    G.dprev = A.d1_prev + (size_t)f * A.d1_frame;
    G.dcur = A.d1_cur + (size_t)f * A.d1_frame;
    G.post = A.d1post ? A.d1post + (size_t)f * A.psi_frame : nullptr;
    G.Z = (unsigned)c.Z;
    G.Wm1 = (unsigned)c.W - 1;
    const unsigned wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const unsigned p = tile * kBlock + threadIdx.x;
    const unsigned w = tile * 4u + wave;
    const float tv = at(G.tot + (unsigned)own, p);
    float psum = 0.0f;
    uint32_t bad = 0;
    if ((tile + 1) * kBlock <= G.Z) {
        group_rows<MODE, Msg, true>(G, nrows, tv, p, w, psum, bad, PK);
        at(A.part + (size_t)f * A.part_frame + (size_t)g * c.Zp, p) = psum;
    } else {
        group_rows<MODE, Msg, false>(G, nrows, tv, p, w, psum, bad, PK);
        if (p < G.Z) at(A.part + (size_t)f * A.part_frame + (size_t)g * c.Zp, p) = psum;
    }
    if (A.vote) vote_store(flag, seen, bad != 0u);
}

struct VnArgs {
    const float *llr;
    const void *msg;
    const float *part;         // owner-group partials, or null: rebuilt from the messages
    float *tot;
    const int32_t *fail;
    size_t msg_frame, tot_frame, part_frame;
    int F, t;
};

// Variable pass layout: the 4 waves of a workgroup split the blocks of one
// core column into kVnGroups row groups, and each group's waves cover
// kVnLanes variables (kVnLanes * VPT with VPT variables per thread), so that
// every wave has one group's loads in flight at once instead of running the
// whole column as a chain of dependent batches.
constexpr int kVnGroups = 2;  // measured: 2 groups of 128 variables beat 1 x 256 and 4 x 64
constexpr int kVnLanes = kBlock / kVnGroups;
// Variables per thread (VPT) of the single-call decoder: 2, so that every
// thread has a whole row group's loads for two variables in flight (measured:
// the variable pass of the rate-0.02 template at Z = 6667 takes 8.2 us for 8
// frames with 2, 9.4 us with 1).
template <typename Msg> constexpr int vn_vpt() { return 2; }
inline unsigned variable_tiles(int Z, int vpt) {
    const int v = kVnLanes * vpt;
    return (unsigned)((Z + v - 1) / v);
}

// Loads per row group and variable issued together: ceil(n / groups) for a
// column of n terms, rounded up to an instantiated width (a longer group
// takes several batches).
inline int variable_group(int max_deg) {
    const int g = ((max_deg > 0 ? max_deg : 1) + kVnGroups - 1) / kVnGroups;
    for (int w : {4, 8, 13, 16, 26})
        if (g <= w) return w;
    return 26;
}

// L = (Q log2(e) + S0) + S1 ...: the product rounded on its own (never fused
// into the first addition), so every schedule that sums the same groups
// gets the same bits.
__device__ __forceinline__ float core_total(float q, const float (&part)[kVnGroups]) {
#pragma clang fp contract(off)
    float L = q * kLog2e;
#pragma unroll
    for (int g = 0; g < kVnGroups; ++g) L += part[g];
    return L;
}

// Step 3 for the core columns: L_v = Q_v + sum of the column's messages (in
// base 2: Q_v log2(e) plus the base-2 messages), in the column's fixed
// summation order: the terms are the owner-group partials P_0 .. P_{G-1}
// followed by the messages of the column's other blocks; row group g of the
// workgroup sums terms [g h, (g + 1) h), h = ceil(terms / 2), in order from
// +0; the group sums meet in LDS and L = (Q + S0) + S1.  kPart: the partials
// come from the check pass (A.part); otherwise each is rebuilt from the
// group's messages, summed in row order from +0, which gives the same bits.
// Messages of block (r, c) with shift s sit at (j - s) mod Z.
template <int G, typename Msg, int VPT, bool kPart>
__device__ __forceinline__ void variable_work(const CodeDev &c, const VnArgs &A, int f, int k,
                                              unsigned tile) {
    constexpr int kWavesPerGroup = kBlock / 64 / kVnGroups;
    constexpr int V = kVnLanes * VPT;  // variables per workgroup
    constexpr int kPB = 4;             // partial loads in flight together
    __shared__ float part[kVnGroups][V];
    const unsigned Z = (unsigned)c.Z;
    const int w = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    const int grp = w / kWavesPerGroup;
    const unsigned v0 = (unsigned)(w % kWavesPerGroup) * 64 + (threadIdx.x & 63);
    unsigned j[VPT], jl[VPT];
#pragma unroll
    for (int e = 0; e < VPT; ++e) {
        j[e] = tile * V + v0 + e * kVnLanes;
        jl[e] = j[e] < Z ? j[e] : Z - 1;  // padding lanes load in range
    }
    const Msg *msg = reinterpret_cast<const Msg *>(A.msg) + (size_t)f * A.msg_frame;
    const int deg = c.core_deg[k];
    const int own = c.core_own[k], ng = c.core_ngrp[k];
    const int terms = ng + deg - own;
    const int half = (terms + 1) / 2;
    const int t0 = grp * half, t1 = min(terms, t0 + half);
    const int32_t *tab = c.core_tab + (size_t)k * c.core_tab_stride;
    // group 0 also reads Q, issued with its first loads
    const float *llr = A.llr + (size_t)f * c.n + (size_t)c.core_col[k] * Z;
    float q[VPT], p[VPT];
#pragma unroll
    for (int e = 0; e < VPT; ++e) {
        q[e] = (grp == 0) ? at(llr, jl[e]) : 0.0f;
        p[e] = 0.0f;
    }
    // The first batch of message terms (table entries [b0, b1)) is loaded
    // first, then the partial terms [t0, pe) are loaded and summed, then the
    // messages are added: the loads of both kinds are in flight together, and
    // the sum keeps the term order.
    const int pe = min(t1, ng);
    const int b0 = own + max(t0, ng) - ng, b1 = own + max(t1, ng) - ng;
    float x[VPT][G];
    if (b0 < b1) {
#pragma unroll
        for (int u = 0; u < G; ++u) {
            const int i = min(b0 + u, b1 - 1);
            const unsigned s = (unsigned)tab[2 * i + 1];
            const Msg *blk = msg + (unsigned)tab[2 * i];
#pragma unroll
            for (int e = 0; e < VPT; ++e) {
                const unsigned idx = (jl[e] >= s) ? jl[e] - s : jl[e] + Z - s;
                x[e][u] = msg_load<Msg>(&at(blk, idx));
            }
        }
    }
    if constexpr (kPart) {
        const float *pp = A.part + (size_t)f * A.part_frame + (size_t)c.core_grp0[k] * c.Zp;
        for (int t = t0; t < pe; t += kPB) {
            float xq[VPT][kPB];
#pragma unroll
            for (int u = 0; u < kPB; ++u) {
                const unsigned row = (unsigned)min(t + u, pe - 1) * (unsigned)c.Zp;
#pragma unroll
                for (int e = 0; e < VPT; ++e) xq[e][u] = at(pp, row + jl[e]);
            }
#pragma unroll
            for (int e = 0; e < VPT; ++e)
#pragma unroll
                for (int u = 0; u < kPB; ++u) p[e] += (t + u < pe) ? xq[e][u] : 0.0f;
        }
    } else {
        for (int t = t0; t < pe; ++t) {
            const int c0 = t * kGroupRows, c1 = min(own, c0 + kGroupRows);
            float xq[VPT][kGroupRows];
#pragma unroll
            for (int u = 0; u < kGroupRows; ++u) {
                const int i = min(c0 + u, c1 - 1);
                const unsigned s = (unsigned)tab[2 * i + 1];
                const Msg *blk = msg + (unsigned)tab[2 * i];
#pragma unroll
                for (int e = 0; e < VPT; ++e) {
                    const unsigned idx = (jl[e] >= s) ? jl[e] - s : jl[e] + Z - s;
                    xq[e][u] = msg_load<Msg>(&at(blk, idx));
                }
            }
#pragma unroll
            for (int e = 0; e < VPT; ++e) {
                float sg = 0.0f;
#pragma unroll
                for (int u = 0; u < kGroupRows; ++u) sg += (c0 + u < c1) ? xq[e][u] : 0.0f;
                p[e] += sg;
            }
        }
    }
    if (b0 < b1) {
#pragma unroll
        for (int e = 0; e < VPT; ++e)
#pragma unroll
            for (int u = 0; u < G; ++u) p[e] += (b0 + u < b1) ? x[e][u] : 0.0f;
    }
    // further batches of message terms
    for (int b = b0 + G; b < b1; b += G) {
#pragma unroll
        for (int u = 0; u < G; ++u) {
            const int i = min(b + u, b1 - 1);
            const unsigned s = (unsigned)tab[2 * i + 1];
            const Msg *blk = msg + (unsigned)tab[2 * i];
#pragma unroll
            for (int e = 0; e < VPT; ++e) {
                const unsigned idx = (jl[e] >= s) ? jl[e] - s : jl[e] + Z - s;
                x[e][u] = msg_load<Msg>(&at(blk, idx));
            }
        }
#pragma unroll
        for (int e = 0; e < VPT; ++e)
#pragma unroll
            for (int u = 0; u < G; ++u) p[e] += (b + u < b1) ? x[e][u] : 0.0f;
    }
#pragma unroll
    for (int e = 0; e < VPT; ++e) part[grp][v0 + e * kVnLanes] = p[e];
    __syncthreads();
    if (grp == 0) {
        float *row = A.tot + (size_t)f * A.tot_frame + (size_t)k * c.Zt;
#pragma unroll
        for (int e = 0; e < VPT; ++e) {
            if (j[e] >= Z) continue;
            float ps[kVnGroups];
#pragma unroll
            for (int g2 = 0; g2 < kVnGroups; ++g2) ps[g2] = part[g2][v0 + e * kVnLanes];
            const float L = core_total(q[e], ps);
            at(row, j[e]) = L;
            at(row, j[e] + Z) = L;
        }
    }
}

// The set-up steps below take kSetupPerThread positions per thread (256
// apart), all loads issued before the first use; a row or column of Z
// positions takes setup_tiles(Z) workgroups.
constexpr int kSetupPerThread = 4;
inline unsigned setup_tiles(int Z) {
    return (unsigned)((Z + kBlock * kSetupPerThread - 1) / (kBlock * kSetupPerThread));
}

// Pack the syndrome bytes into 64-bit words per base row: bit a%64 of word a/64,
// for check a of the relabelled row.
__device__ __forceinline__ void pack_syndrome_work(const CodeDev &c, const uint8_t *syn,
                                                   uint64_t *synbits, size_t syn_frame, int f, int r,
                                                   unsigned tile) {
    const int Z = c.Z;
    const int rot = c.row_rot[r];
    const uint8_t *row = syn + (size_t)f * c.m + (size_t)r * Z;
    int v[kSetupPerThread];
#pragma unroll
    for (int q = 0; q < kSetupPerThread; ++q) {
        const int a = (int)((tile * kSetupPerThread + q) * kBlock + threadIdx.x);
        int j = a - rot;  // the check's index in the code as given
        j += (j < 0) ? Z : 0;
        v[q] = a < Z ? (row[j] & 1) : 0;
    }
#pragma unroll
    for (int q = 0; q < kSetupPerThread; ++q) {
        const int a = (int)((tile * kSetupPerThread + q) * kBlock + threadIdx.x);
        const unsigned long long bits = wave_ballot(v[q] != 0);
        if ((threadIdx.x & 63) == 0 && a < Z)
            synbits[(size_t)f * syn_frame + (size_t)r * c.W + (a >> 6)] = bits;
    }
}

// Core totals of iteration 0: L_v = Q_v, in base 2 (both copies of the row).
__device__ __forceinline__ void init_totals_work(const CodeDev &c, const float *llr, float *tot,
                                                 size_t tot_frame, int f, int k, unsigned tile) {
    const float *src = llr + (size_t)f * c.n + (size_t)c.core_col[k] * c.Z;
    float *row = tot + (size_t)f * tot_frame + (size_t)k * c.Zt;
    float q[kSetupPerThread];
#pragma unroll
    for (int u = 0; u < kSetupPerThread; ++u) {
        const int j = (int)((tile * kSetupPerThread + u) * kBlock + threadIdx.x);
        q[u] = j < c.Z ? src[j] * kLog2e : 0.0f;
    }
#pragma unroll
    for (int u = 0; u < kSetupPerThread; ++u) {
        const int j = (int)((tile * kSetupPerThread + u) * kBlock + threadIdx.x);
        if (j < c.Z) {
            row[j] = q[u];
            row[j + c.Z] = q[u];
        }
    }
}

// Degree-1 inputs in check order: Psi[a] = d1_input(Q_p), p the variable of
// check a of degree-1 block k (+-Phi(|Q_p|), or +-e^{-|Q_p|} where the block's
// row is updated in the t-domain), once per decode.
__device__ __forceinline__ void init_psi_work(const CodeDev &c, const float *llr, float *psi,
                                              size_t psi_frame, int f, int k, unsigned tile) {
    const unsigned Z = (unsigned)c.Z;
    const unsigned s = (unsigned)c.d1_shift[k];
    const bool tdom = c.d1_tdom[k] != 0;
    const float *src = llr + (size_t)f * c.n + (size_t)c.d1_col[k] * Z;
    float *dst = psi + (size_t)f * psi_frame + (size_t)k * c.Zp;
    const PhiConsts PK = phi_consts();
    float q[kSetupPerThread];
#pragma unroll
    for (int u = 0; u < kSetupPerThread; ++u) {
        const unsigned a = (tile * kSetupPerThread + u) * kBlock + threadIdx.x;
        unsigned j = a + s;
        j -= (j >= Z) ? Z : 0u;
        q[u] = a < Z ? src[j] : 0.0f;
    }
#pragma unroll
    for (int u = 0; u < kSetupPerThread; ++u) {
        const unsigned a = (tile * kSetupPerThread + u) * kBlock + threadIdx.x;
        if (a < Z) dst[a] = d1_input(q[u], tdom, PK);
    }
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
// the exit iteration, for positions tile 256 + thread of base column col.  The
// channel LLR is read only where it decides: degree-0 columns, degree-1
// columns at t = 0, and posteriors at t = 0.
__device__ __forceinline__ void finalize_work(const CodeDev &c, const FinArgs &A, int f, int col,
                                              unsigned tile) {
    const int Z = c.Z;
    const int j = (int)(tile * kBlock + threadIdx.x);
    if (j >= Z) return;
    const int it = uniform_i32(A.iters_out + f);
    const int kind = uniform_i32(c.col_kind + col), ref = uniform_i32(c.col_ref + col);
    const size_t v = (size_t)f * c.n + (size_t)col * Z + j;
    int bit;
    float L = 0.0f;
    if (kind == COL_CORE) {
        const float Lb = A.tot[(size_t)f * A.tot_frame + (size_t)ref * c.Zt + j];
        bit = Lb < 0.0f;  // at t = 0 the totals are Q log2(e): the sign of Q
        if (A.llr_out) L = it > 0 ? Lb * kLn2 : A.llr[v];  // at t = 0 the posterior is Q itself
    } else if (kind == COL_DEG1 && it > 0) {
        int a = j - c.d1_shift[ref];
        a += (a < 0) ? Z : 0;
        const uint64_t wd = A.d1bits[it & 1][(size_t)f * A.d1_frame + (size_t)ref * c.W + (a >> 6)];
        bit = (int)((wd >> (a & 63)) & 1ull);
        if (A.llr_out) L = A.d1post[it & 1][(size_t)f * A.psi_frame + (size_t)ref * c.Zp + a];
    } else {
        L = A.llr[v];
        bit = L < 0.0f;
    }
    A.bits_out[v] = (uint8_t)bit;
    if (A.llr_out) A.llr_out[v] = L;
}


}  // namespace dev
}  // namespace ldpc
