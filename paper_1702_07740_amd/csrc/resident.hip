// Frame-resident decoder, gfx950: one workgroup decodes one frame for all of
// its iterations in a single launch, with the frame's whole decode state in
// LDS.
//
// For small liftings the per-iteration launches of the flooding schedule
// (decoder.hip) are bound by launch latency, not by work: each pass over a
// code of n = 9,600 takes a few microseconds whatever it computes.  Here a
// frame's check-to-variable messages, core totals, packed syndrome and
// degree-1 decision bits live in LDS (160 KB per CU), the iteration loop runs
// inside the kernel, and the only synchronisation is the workgroup barrier
// between the phases of an iteration: the check phase (Alg. 1 Step 2, with
// the Step 4 check of the previous iteration), the row-group sums of the
// variable phase (Step 3), and the core totals.  Global memory is
// touched only to read the channel LLRs, to hold the degree-1 inputs Psi
// (read-only after the first phase), and to write the outputs.
//
// The arithmetic is the per-iteration decoder's, operation for operation: the
// same base-2 state, the same phi2 and t-domain check update, the same
// prefix/suffix order of the exclusive sums, the same degree-1 decisions, and
// core totals
// summed as (Q + S0) + S1 over the same two row groups.  So a frame decodes to
// the same bits, iteration count and convergence flag on either schedule.
//
// Two simplifications against the per-iteration decoder, both exact:
//  - messages start at zero in LDS, so the first iteration is a steady one
//    (L_v - 0 = L_v);
//  - the decision bits of iteration 0 for the degree-1 variables (the channel
//    signs, in check order) are written once at set-up, so the first
//    iteration and a zero-iteration decode read them like any other.
#include "passes.h"

namespace ldpc {

namespace {

using namespace dev;

constexpr int kResThreads = 1024;  // 16 wave64s: four per SIMD of the one CU

template <typename Msg>
struct ResView {
    Msg *msg;            // [NS][Z] messages, check order (LDS), written by the check phase
    const Msg *msg_in;   // where the check phase reads the previous messages (= msg here;
                         // the other buffer of a pair in the frame-split schedule)
    float *tot;          // [NC][Z] core totals, base 2 (LDS)
    const float *q;      // [NC][Z] channel LLRs of the core variables (LDS)
    const uint64_t *syn; // [mb][W] packed syndrome bits (LDS)
    const float *psi;    // [ND1][Zp] +-Phi(|Q|) of the degree-1 variables, check order (global)
    unsigned Z, W, Zp;
};

// K units of a common row class (degree D, DS stored blocks, then one
// degree-1 block if DS < D): for each q < K, checks ch[q]*64 + lane of the
// row whose resident descriptor is d[q].  The K units' loads issue together,
// so a wave has K independent chains in flight.  UPDATE = false only votes.
// Returns true if one of the lane's checks fails the parity check of the
// voted decisions (core: sign of the totals read; degree-1: dprev).
template <int D, int DS, bool UPDATE, typename Msg, int K>
__device__ __forceinline__ bool res_fixed(const ResView<Msg> &S, const int32_t *const (&d)[K],
                                          const unsigned (&ch)[K], const uint64_t *dprev,
                                          uint64_t *dcur, const PhiConsts &PK) {
    const unsigned Z = S.Z, lane = threadIdx.x & 63u;
    float x[K][D];
    bool dec[K][D];
    unsigned idx[K][D];  // stored: message index; degree-1: decision-word index
    uint64_t sw[K];
    bool valid[K];
#pragma unroll
    for (int q = 0; q < K; ++q) {
        const unsigned a = ch[q] * 64u + lane;
        valid[q] = a < Z;
        const unsigned al = valid[q] ? a : Z - 1;
        sw[q] = S.syn[(unsigned)uniform_i32(d[q] + 4) + ch[q]];
#pragma unroll
        for (int k = 0; k < D; ++k) {
            const unsigned s = (unsigned)uniform_i32(d[q] + 17 + k);
            const unsigned o0 = (unsigned)uniform_i32(d[q] + 5 + k);
            const unsigned o1 = (unsigned)uniform_i32(d[q] + 11 + k);
            if (k < DS) {
                unsigned j = al + s;
                j -= (j >= Z) ? Z : 0u;
                const float lt = S.tot[o0 + j];
                idx[q][k] = o1 + a;
                const float mo = UPDATE ? msg_load<Msg>(&S.msg_in[o1 + al]) : 0.0f;
                x[q][k] = lt - mo;
                dec[q][k] = lt < 0.0f;
            } else {
                x[q][k] = S.psi[o0 + al];
                idx[q][k] = o1 + ch[q];
                dec[q][k] = (dprev[idx[q][k]] >> lane) & 1ull;
            }
        }
    }
    bool bad = false;
#pragma unroll
    for (int q = 0; q < K; ++q) {
        bool par = (sw[q] >> lane) & 1ull;
#pragma unroll
        for (int k = 0; k < D; ++k) par ^= dec[q][k];
        bad |= par && valid[q];
    }
    if (!UPDATE) return bad;

#pragma unroll
    for (int q = 0; q < K; ++q) {
        if constexpr (D == 3 && DS == 2) {
            // Step 2 in the t-domain, as in the per-iteration check pass
            bool neg[3];
            bool p2 = (sw[q] >> lane) & 1ull;
#pragma unroll
            for (int k = 0; k < 3; ++k) {
                neg[k] = x[q][k] < 0.0f;
                p2 ^= neg[k];
            }
            float mag[2], t1, t2;
            bool q_wins;
            tdom_check3(x[q][0], x[q][1], fabsf(x[q][2]), PK, mag[0], mag[1], q_wins, t1, t2);
#pragma unroll
            for (int k = 0; k < 2; ++k)
                if (valid[q]) msg_store<Msg>(&S.msg[idx[q][k]], (p2 ^ neg[k]) ? -mag[k] : mag[k]);
            const bool dd = neg[2] ^ (p2 && !q_wins);
            const unsigned long long bits = wave_ballot(valid[q] && dd);
            if (lane == 0) dcur[idx[q][2]] = bits;
            continue;
        }
        // Step 2: sign product with the syndrome bit, Phi-domain exclusive sums
        float ph[D], ex[D];
        bool neg[D];
        const bool p2 = phi_exclusive<D, DS>(x[q], (sw[q] >> lane) & 1ull, PK, neg, ph, ex);
#pragma unroll
        for (int k = 0; k < D; ++k) {
            const bool sgn = p2 ^ neg[k];  // the message to block k is negative
            if (k < DS) {
                const float mag = phi2(ex[k], PK);
                if (valid[q]) msg_store<Msg>(&S.msg[idx[q][k]], sgn ? -mag : mag);
            } else {
                const bool dd = d1_decision(neg[k], p2, ph[k], ex[k], PK);
                const unsigned long long bits = wave_ballot(valid[q] && dd);
                if (lane == 0) dcur[idx[q][k]] = bits;
            }
        }
    }
    return bad;
}

// One unit of any other row (degree up to D, stored count and degree read at
// run time), offsets from the block tables; same arithmetic as above.
template <int D, bool UPDATE, typename Msg>
__device__ __forceinline__ bool res_generic(const CodeDev &c, const ResView<Msg> &S,
                                            const int32_t *d, unsigned ch, const uint64_t *dprev,
                                            uint64_t *dcur, const PhiConsts &PK) {
    const unsigned Z = S.Z, lane = threadIdx.x & 63u;
    const unsigned a = ch * 64u + lane;
    const bool valid = a < Z;
    const unsigned al = valid ? a : Z - 1;
    const int deg = uniform_i32(d + 1);
    const int ns = uniform_i32(d + 2);
    const int b0 = uniform_i32(d + 3);
    const uint64_t sw = S.syn[(unsigned)uniform_i32(d + 4) + ch];
    float x[D];
    bool dec[D];
    unsigned idx[D];
#pragma unroll
    for (int k = 0; k < D; ++k) {
        x[k] = 0.0f;
        dec[k] = false;
        idx[k] = 0;
        if (k >= deg) continue;
        const int b = b0 + k;
        const unsigned s = (unsigned)uniform_i32(c.blk_shift + b);
        const unsigned ref = (unsigned)uniform_i32(c.blk_ref + b);
        if (k < ns) {
            unsigned j = al + s;
            j -= (j >= Z) ? Z : 0u;
            const float lt = S.tot[(unsigned)uniform_i32(c.blk_core + b) * Z + j];
            idx[k] = ref * Z + a;
            const float mo = UPDATE ? msg_load<Msg>(&S.msg_in[ref * Z + al]) : 0.0f;
            x[k] = lt - mo;
            dec[k] = lt < 0.0f;
        } else {
            x[k] = S.psi[ref * S.Zp + al];
            idx[k] = ref * S.W + ch;
            dec[k] = (dprev[idx[k]] >> lane) & 1ull;
        }
    }
    bool par = (sw >> lane) & 1ull;
#pragma unroll
    for (int k = 0; k < D; ++k) par ^= dec[k];
    const bool bad = par && valid;
    if (!UPDATE) return bad;

    float ph[D];
    bool neg[D];
    bool p2 = (sw >> lane) & 1ull;
#pragma unroll
    for (int k = 0; k < D; ++k) {
        ph[k] = 0.0f;
        neg[k] = false;
        if (k >= deg) continue;
        neg[k] = x[k] < 0.0f;
        p2 ^= neg[k];
        ph[k] = (k < ns) ? phi2(fabsf(x[k]), PK) : fabsf(x[k]);
    }
    // exclusive sums over the first deg entries: the same additions as the
    // fixed-degree form (adding the initial 0 is exact)
    float ex[D];
    float pre[D];
    pre[0] = 0.0f;
#pragma unroll
    for (int k = 1; k < D; ++k) pre[k] = pre[k - 1] + ph[k - 1];
    float suf = 0.0f;
#pragma unroll
    for (int k = D - 1; k >= 0; --k) {
        ex[k] = 0.0f;
        if (k >= deg) continue;
        ex[k] = pre[k] + suf;
        suf += ph[k];
    }
#pragma unroll
    for (int k = 0; k < D; ++k) {
        if (k >= deg) continue;
        const bool sgn = p2 ^ neg[k];
        if (k < ns) {
            const float mag = phi2(ex[k], PK);
            if (valid) msg_store<Msg>(&S.msg[idx[k]], sgn ? -mag : mag);
        } else {
            const bool dd = d1_decision(neg[k], p2, ph[k], ex[k], PK);
            const unsigned long long bits = wave_ballot(valid && dd);
            if (lane == 0) dcur[idx[k]] = bits;
        }
    }
    return bad;
}

// One unit (row descriptor d, chunk ch) of any class (GENERIC = false: the
// code has common rows only).
template <bool UPDATE, typename Msg, bool GENERIC>
__device__ __forceinline__ bool res_unit(const CodeDev &c, const ResView<Msg> &S, int cls,
                                         const int32_t *d, unsigned ch, const uint64_t *dprev,
                                         uint64_t *dcur, const PhiConsts &PK) {
    const int32_t *const dv[1] = {d};
    const unsigned cv[1] = {ch};
#define LDPC_RES(I, D, DS) \
    case I: return res_fixed<D, DS, UPDATE, Msg, 1>(S, dv, cv, dprev, dcur, PK);
    switch (cls) {
        LDPC_RES(0, 1, 0) LDPC_RES(1, 1, 1) LDPC_RES(2, 2, 1) LDPC_RES(3, 2, 2)
        LDPC_RES(4, 3, 2) LDPC_RES(5, 3, 3) LDPC_RES(6, 4, 3) LDPC_RES(7, 4, 4)
        LDPC_RES(8, 5, 4) LDPC_RES(9, 5, 5) LDPC_RES(10, 6, 5) LDPC_RES(11, 6, 6)
        default: break;
    }
#undef LDPC_RES
    if constexpr (GENERIC) {
        if (cls == 12) return res_generic<8, UPDATE, Msg>(c, S, d, ch, dprev, dcur, PK);
        if (cls == 13) return res_generic<16, UPDATE, Msg>(c, S, d, ch, dprev, dcur, PK);
    }
    return false;
}

// Check phase of one frame.  The units (row, chunk of 64 checks) are listed
// with the rows in class order; the frame's waves (wave index `wave` of `nw`,
// across all of the frame's workgroups) take pairs of consecutive units in
// turn, and a pair of one common class runs as one two-unit chain.  A unit's
// messages and decision word belong to one wave for the whole decode.
template <bool UPDATE, typename Msg, bool GENERIC>
__device__ __forceinline__ bool res_check_phase(const CodeDev &c, const ResView<Msg> &S,
                                                const uint64_t *dprev, uint64_t *dcur,
                                                const PhiConsts &PK, int wave, int nw) {
    const int units = c.res_units;
    bool bad = false;
    for (int u = 2 * wave; u < units; u += 2 * nw) {
        const bool two = u + 1 < units;
        const int32_t pk0 = uniform_i32(c.res_unit + u);
        const int32_t pk1 = uniform_i32(c.res_unit + (two ? u + 1 : u));
        const int32_t *const d[2] = {c.res_desc + (size_t)(pk0 & 0xffff) * kResDescWords,
                                     c.res_desc + (size_t)(pk1 & 0xffff) * kResDescWords};
        const unsigned ch[2] = {(unsigned)pk0 >> 16, (unsigned)pk1 >> 16};
        const int cls0 = uniform_i32(d[0]), cls1 = uniform_i32(d[1]);
        if (two && cls0 == cls1 && cls0 < kFixedClasses) {
#define LDPC_RES2(I, D, DS) \
    case I: bad |= res_fixed<D, DS, UPDATE, Msg, 2>(S, d, ch, dprev, dcur, PK); break;
            switch (cls0) {
                LDPC_RES2(0, 1, 0) LDPC_RES2(1, 1, 1) LDPC_RES2(2, 2, 1) LDPC_RES2(3, 2, 2)
                LDPC_RES2(4, 3, 2) LDPC_RES2(5, 3, 3) LDPC_RES2(6, 4, 3) LDPC_RES2(7, 4, 4)
                LDPC_RES2(8, 5, 4) LDPC_RES2(9, 5, 5) LDPC_RES2(10, 6, 5) LDPC_RES2(11, 6, 6)
                default: break;
            }
#undef LDPC_RES2
        } else {
            bad |= res_unit<UPDATE, Msg, GENERIC>(c, S, cls0, d[0], ch[0], dprev, dcur, PK);
            if (two)
                bad |= res_unit<UPDATE, Msg, GENERIC>(c, S, cls1, d[1], ch[1], dprev, dcur, PK);
        }
    }
    return bad;
}

// Variable phase, first half: the row-group sums S0 and S1 of every core
// variable, in the column's summation order (the owner-group partials, each
// rebuilt from its messages in row order from +0, then the other blocks'
// messages; S0 the first ceil(terms / 2) terms, S1 the rest, each from +0),
// as in the per-iteration decoder, one wave per (column, 64 variables,
// group), into part[g].
template <typename Msg>
__device__ __forceinline__ void res_group_sums(const CodeDev &c, const ResView<Msg> &S,
                                               float *const *part) {
    const unsigned nw = blockDim.x >> 6;
    const unsigned wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const unsigned Z = S.Z, units = (unsigned)c.NC * S.W * kVnGroups;
    for (unsigned u = wave; u < units; u += nw) {
        const int g = (int)(u % kVnGroups);
        const unsigned kc = u / kVnGroups;
        const int k = (int)(kc / S.W);
        const unsigned jv = (kc - (unsigned)k * S.W) * 64u + (threadIdx.x & 63u);
        // every lane stays active through the loads (the table window is one
        // pair per lane); lanes past Z read variable Z - 1 and store nothing
        const bool valid = jv < Z;
        const unsigned j = valid ? jv : Z - 1;
        const int deg = uniform_i32(c.core_deg + k);
        const int own = uniform_i32(c.core_own + k), ng = uniform_i32(c.core_ngrp + k);
        const int terms = ng + deg - own;
        const int per = (terms + kVnGroups - 1) / kVnGroups;
        const int t0 = g * per, t1 = min(terms, t0 + per);
        const int32_t *tab = c.res_core + (size_t)k * c.res_core_stride;
        // The column's (offset, shift) pairs, 64 at a time, one per lane
        // (one vector load instead of a chain of scalar loads); a block's
        // pair is then read from its lane.
        int w0 = -(1 << 30), voff = 0, vsh = 0;
        auto window = [&](int lo, int hi) {  // make pairs [lo, hi) readable, hi - lo <= 64
            if (lo < w0 || hi > w0 + 64) {
                w0 = lo;
                const int e = w0 + (int)(threadIdx.x & 63u);
                voff = e < deg ? tab[2 * e] : 0;
                vsh = e < deg ? tab[2 * e + 1] : 0;
            }
        };
        auto load = [&](int i) {
            const unsigned off = (unsigned)__builtin_amdgcn_readlane(voff, i - w0);
            const unsigned s = (unsigned)__builtin_amdgcn_readlane(vsh, i - w0);
            const unsigned idx = (j >= s) ? j - s : j + Z - s;
            return msg_load<Msg>(&S.msg[off + idx]);
        };
        float p = 0.0f;
        // partial terms: each group's owned messages, summed from +0
        for (int t = t0; t < min(t1, ng); ++t) {
            const int b0 = t * kGroupRows, b1 = min(own, b0 + kGroupRows);
            window(b0, b0 + kGroupRows);
            float xv[kGroupRows];
#pragma unroll
            for (int u2 = 0; u2 < kGroupRows; ++u2) xv[u2] = load(min(b0 + u2, b1 - 1));
            float sg = 0.0f;
#pragma unroll
            for (int u2 = 0; u2 < kGroupRows; ++u2) sg += (b0 + u2 < b1) ? xv[u2] : 0.0f;
            p += sg;
        }
        // message terms: table entries [own + max(t0, ng) - ng, own + max(t1, ng) - ng),
        // in batches of kResVnBatch blocks: one burst of table loads, then
        // their LDS loads together.  Entries past the range (valid offsets:
        // the table is padded) add +0, which leaves a sum that started at +0
        // unchanged.
        const int e = own + max(t1, ng) - ng;
        for (int i0 = own + max(t0, ng) - ng; i0 < e; i0 += kResVnBatch) {
            window(i0, i0 + kResVnBatch);
            float xv[kResVnBatch];
#pragma unroll
            for (int u2 = 0; u2 < kResVnBatch; ++u2) xv[u2] = load(i0 + u2);
#pragma unroll
            for (int u2 = 0; u2 < kResVnBatch; ++u2) p += (i0 + u2 < e) ? xv[u2] : 0.0f;
        }
        if (valid) part[g][(unsigned)k * Z + j] = p;
    }
}

// Variable phase, second half (after a barrier): L_v = (Q_v log2(e) + S0) + S1.
template <typename Msg>
__device__ __forceinline__ void res_totals(const CodeDev &c, const ResView<Msg> &S,
                                           float *const *part) {
    const unsigned n = (unsigned)c.NC * S.Z;
    for (unsigned i = threadIdx.x; i < n; i += blockDim.x) {
        float ps[kVnGroups];
#pragma unroll
        for (int g = 0; g < kVnGroups; ++g) ps[g] = part[g][i];
        S.tot[i] = core_total(S.q[i], ps);
    }
}

// kGeneric: the code has rows outside the common classes (degree > 6, or more
// than one degree-1 block).  Their code path holds many more registers, so
// codes without such rows run an instantiation that leaves it out.
template <typename Msg, bool kGeneric>
__global__ __launch_bounds__(kResThreads) void resident_decode(CodeDev c, ResidentArgs A) {
    extern __shared__ __attribute__((aligned(16))) unsigned char lds[];
    const int f = blockIdx.x;
    const unsigned Z = (unsigned)c.Z, W = (unsigned)c.W, Zp = (unsigned)c.Zp;
    ResView<Msg> S;
    S.msg = reinterpret_cast<Msg *>(lds);
    S.msg_in = S.msg;
    S.tot = reinterpret_cast<float *>(lds + A.lds_tot);
    float *qc = reinterpret_cast<float *>(lds + A.lds_q);
    S.q = qc;
    float *part[kVnGroups];  // the row-group sums, NC * Z each
#pragma unroll
    for (int g = 0; g < kVnGroups; ++g)
        part[g] = reinterpret_cast<float *>(lds + A.lds_part) + (size_t)g * c.NC * c.Z;
    uint64_t *syn = reinterpret_cast<uint64_t *>(lds + A.lds_syn);
    S.syn = syn;
    uint64_t *d1 = reinterpret_cast<uint64_t *>(lds + A.lds_d1);  // [2][ND1][W]
    int32_t *flag = reinterpret_cast<int32_t *>(lds + A.lds_flag); // [2]
    float *psi = A.psi + (size_t)f * A.psi_frame;
    S.psi = psi;
    S.Z = Z;
    S.W = W;
    S.Zp = Zp;
    const float *llr = A.llr + (size_t)f * c.n;
    const uint8_t *syn_in = A.syndrome + (size_t)f * c.m;
    const size_t d1n = (size_t)c.ND1 * W;
    const unsigned nt = blockDim.x, nw = nt >> 6, lane = threadIdx.x & 63u;
    const unsigned wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const PhiConsts PK = phi_consts();

    // Set-up: zero messages, the core LLRs and the totals of iteration 0, Psi
    // and the channel-sign decision bits of the degree-1 variables, packed
    // syndrome, vote flags.
    for (unsigned i = threadIdx.x; i < (unsigned)c.NS * Z; i += nt) msg_store<Msg>(&S.msg[i], 0.0f);
    for (unsigned i = threadIdx.x; i < (unsigned)c.NC * Z; i += nt) {
        const unsigned k = i / Z, j = i - k * Z;
        const float q = llr[(size_t)c.core_col[k] * Z + j];
        qc[i] = q;
        S.tot[i] = q * kLog2e;
    }
    for (unsigned u = wave; u < (unsigned)c.ND1 * W; u += nw) {
        const unsigned k = u / W, a = (u - k * W) * 64u + lane;
        bool neg = false;
        if (a < Z) {
            unsigned j = a + (unsigned)uniform_i32(c.d1_shift + k);
            j -= (j >= Z) ? Z : 0u;
            const float q = llr[(size_t)uniform_i32(c.d1_col + k) * Z + j];
            psi[k * Zp + a] = d1_input(q, uniform_i32(c.d1_tdom + k) != 0, PK);
            neg = q < 0.0f;
        }
        const unsigned long long bits = wave_ballot(neg);
        if (lane == 0) d1[u] = bits;
    }
    for (unsigned u = wave; u < (unsigned)c.mb * W; u += nw) {
        const unsigned r = u / W, a = (u - r * W) * 64u + lane;
        // check a of the relabelled row is check (a - rot) mod Z as given
        const unsigned rot = (unsigned)uniform_i32(c.row_rot + r);
        const unsigned jg = (a >= rot) ? a - rot : a + Z - rot;
        const bool v = a < Z && (syn_in[(size_t)r * Z + jg] & 1);
        const unsigned long long bits = wave_ballot(v);
        if (lane == 0) syn[u] = bits;
    }
    if (threadIdx.x < 2) flag[threadIdx.x] = 0;
    __syncthreads();

    const int T = A.T;
    auto checked = [&](int t) { return t == T || (A.early_stop && t >= A.check_from); };
    int it = T, conv = 0;
    bool stopped = false;
    for (int t = 1; t <= T; ++t) {
        const bool vote = checked(t - 1);
        const bool bad = res_check_phase<true, Msg, kGeneric>(c, S, d1 + ((t - 1) & 1) * d1n,
                                                              d1 + (t & 1) * d1n, PK, (int)wave,
                                                              (int)nw);
        if (vote && wave_ballot(bad) != 0ull && lane == 0) flag[t & 1] = 1;
        __syncthreads();
        if (vote && flag[t & 1] == 0) {
            // the decisions of iteration t - 1 satisfy H x = s: stop there
            it = t - 1;
            conv = 1;
            stopped = true;
            break;
        }
        // flag[(t + 1) & 1] was last read before the previous barrier
        if (threadIdx.x == 0) flag[(t + 1) & 1] = 0;
        res_group_sums<Msg>(c, S, part);
        __syncthreads();
        res_totals<Msg>(c, S, part);
        __syncthreads();
    }
    if (!stopped) {
        // the check of the last iteration (the channel decisions when T = 0)
        const bool bad = res_check_phase<false, Msg, kGeneric>(c, S, d1 + (T & 1) * d1n, nullptr,
                                                               PK, (int)wave, (int)nw);
        if (wave_ballot(bad) != 0ull && lane == 0) flag[(T + 1) & 1] = 1;
        __syncthreads();
        conv = flag[(T + 1) & 1] == 0;
    }

    // Read-out: decisions at the exit iteration.
    const uint64_t *dexit = d1 + (it & 1) * d1n;
    uint8_t *bits_out = A.bits_out + (size_t)f * c.n;
    for (unsigned v = threadIdx.x; v < (unsigned)c.n; v += nt) {
        const unsigned col = v / Z, j = v - col * Z;
        const int kind = c.col_kind[col];
        const unsigned ref = (unsigned)c.col_ref[col];
        int bit = llr[v] < 0.0f;
        if (kind == COL_CORE) {
            bit = S.tot[ref * Z + j] < 0.0f;
        } else if (kind == COL_DEG1 && it > 0) {
            unsigned a = j + Z - (unsigned)c.d1_shift[ref];
            a -= (a >= Z) ? Z : 0u;
            bit = (int)((dexit[ref * W + (a >> 6)] >> (a & 63u)) & 1ull);
        }
        bits_out[v] = (uint8_t)bit;
    }
    if (threadIdx.x == 0) {
        A.iters_out[f] = it;
        A.conv_out[f] = (uint8_t)conv;
    }
}

// ---------------------------------------------------------------------------
// Frame-split schedule.  K workgroups share a frame: the check phase's units
// are dealt over all of the frame's waves, and every workgroup recomputes the
// frame's core totals into its own LDS from the messages in global memory
// (the same row-group sums and totals as above, so the same bits).  One
// barrier across the frame's workgroups per iteration separates the check
// phase from the totals.  Messages alternate between two buffers by iteration
// parity: the check phase of iteration t reads the messages of t - 1 from one
// and writes those of t to the other, so a workgroup that starts iteration
// t + 1 while another still sums the messages of t writes only the buffer
// nobody reads.  Everything else the check phase touches (a unit's messages,
// its decision word) belongs to one wave for the whole decode.

constexpr int kSplitThreads = 1024;
constexpr unsigned kSplitSpinLimit = 1u << 22;  // polls of about 60 ns: a quarter second

struct SplitArgs {
    const float *llr;          // [F][n]
    const uint8_t *syndrome;   // [F][m]
    float *psi;                // [F][ND1][Zp]
    void *msg[2];              // two message buffers, [F][NS][Z] each
    uint64_t *synbits;         // [F][mb][W]
    uint64_t *d1[2];           // [F][ND1][W] each, by iteration parity
    int32_t *team;             // [F] arrival counters, then [T + 2][F] vote flags; zero at launch
    uint8_t *bits_out;
    int32_t *iters_out;
    uint8_t *conv_out;
    size_t msg_frame, psi_frame, d1_frame, syn_frame;
    int T, early_stop, check_from, K, F;
    unsigned lds_q, lds_part;  // LDS: totals at 0, core LLRs, row-group sums
};

// Barrier across the workgroups of one frame: every wave's stores leave
// first; one thread publishes them to the device (agent-scope release),
// arrives, waits for all K arrivals of this round (a bounded wait), and makes
// the others' stores visible to the workgroup (agent-scope acquire).  Returns
// false if the wait ran out, which the caller reports as a failed decode.
__device__ __forceinline__ bool team_barrier(int32_t *ctr, int target) {
    __shared__ int ok_s;
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
    if (threadIdx.x == 0) {
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
        __hip_atomic_fetch_add(ctr, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        int ok = 1;
        unsigned n = 0;
        while (__hip_atomic_load(ctr, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < target) {
            __builtin_amdgcn_s_sleep(2);
            if (++n > kSplitSpinLimit) {
                ok = 0;
                break;
            }
        }
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
        ok_s = ok;
    }
    __syncthreads();
    return ok_s != 0;
}

__device__ __forceinline__ int32_t agent_load(const int32_t *p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

template <typename Msg, bool kGeneric>
__global__ __launch_bounds__(kSplitThreads) void split_decode(CodeDev c, SplitArgs A) {
    extern __shared__ __attribute__((aligned(16))) unsigned char lds[];
    // workgroup g: XCD g mod 8 (the hardware's dealing order); the K members
    // of a frame sit on one XCD
    const unsigned g = blockIdx.x, x = g % 8u, j = g / 8u, K = (unsigned)A.K;
    const unsigned k = j % K;
    const int f = (int)(x + 8u * (j / K));
    if (f >= A.F) return;  // padding workgroups of a frame that does not exist
    const unsigned Z = (unsigned)c.Z, W = (unsigned)c.W, Zp = (unsigned)c.Zp;
    const unsigned nt = blockDim.x, nw = nt >> 6, lane = threadIdx.x & 63u;
    const unsigned wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int gw = (int)(k * nw + wave), NW = (int)(K * nw);
    const unsigned gt = k * nt + threadIdx.x, NT = K * nt;
    const PhiConsts PK = phi_consts();
    float *tot = reinterpret_cast<float *>(lds);
    float *qc = reinterpret_cast<float *>(lds + A.lds_q);
    float *part[kVnGroups];  // the row-group sums, NC * Z each
#pragma unroll
    for (int g = 0; g < kVnGroups; ++g)
        part[g] = reinterpret_cast<float *>(lds + A.lds_part) + (size_t)g * c.NC * c.Z;
    Msg *mb[2] = {reinterpret_cast<Msg *>(A.msg[0]) + (size_t)f * A.msg_frame,
                  reinterpret_cast<Msg *>(A.msg[1]) + (size_t)f * A.msg_frame};
    uint64_t *d1[2] = {A.d1[0] + (size_t)f * A.d1_frame, A.d1[1] + (size_t)f * A.d1_frame};
    uint64_t *syn = A.synbits + (size_t)f * A.syn_frame;
    float *psi = A.psi + (size_t)f * A.psi_frame;
    ResView<Msg> S;
    S.msg = mb[1];
    S.msg_in = mb[0];
    S.tot = tot;
    S.q = qc;
    S.syn = syn;
    S.psi = psi;
    S.Z = Z;
    S.W = W;
    S.Zp = Zp;
    int32_t *ctr = A.team + f;
    int32_t *flags = A.team + A.F;  // [T + 2][F]
    const float *llr = A.llr + (size_t)f * c.n;
    const uint8_t *syn_in = A.syndrome + (size_t)f * c.m;
    int epoch = 0;
    bool ok = true;

    // Set-up over the frame's workgroups: messages of iteration 0 (zero), Psi
    // and the channel-sign decision bits of the degree-1 variables, packed
    // syndrome; per workgroup: core LLRs and the totals of iteration 0.
    for (unsigned i = gt; i < (unsigned)c.NS * Z; i += NT) msg_store<Msg>(&mb[0][i], 0.0f);
    for (unsigned u = (unsigned)gw; u < (unsigned)c.ND1 * W; u += (unsigned)NW) {
        const unsigned kk = u / W, a = (u - kk * W) * 64u + lane;
        bool neg = false;
        if (a < Z) {
            unsigned jj = a + (unsigned)uniform_i32(c.d1_shift + kk);
            jj -= (jj >= Z) ? Z : 0u;
            const float q = llr[(size_t)uniform_i32(c.d1_col + kk) * Z + jj];
            psi[kk * Zp + a] = d1_input(q, uniform_i32(c.d1_tdom + kk) != 0, PK);
            neg = q < 0.0f;
        }
        const unsigned long long bits = wave_ballot(neg);
        if (lane == 0) d1[0][u] = bits;
    }
    for (unsigned u = (unsigned)gw; u < (unsigned)c.mb * W; u += (unsigned)NW) {
        const unsigned r = u / W, a = (u - r * W) * 64u + lane;
        const unsigned rot = (unsigned)uniform_i32(c.row_rot + r);
        const unsigned jg = (a >= rot) ? a - rot : a + Z - rot;
        const bool v = a < Z && (syn_in[(size_t)r * Z + jg] & 1);
        const unsigned long long bits = wave_ballot(v);
        if (lane == 0) syn[u] = bits;
    }
    for (unsigned i = threadIdx.x; i < (unsigned)c.NC * Z; i += nt) {
        const unsigned kk = i / Z, jj = i - kk * Z;
        const float q = llr[(size_t)c.core_col[kk] * Z + jj];
        qc[i] = q;
        tot[i] = q * kLog2e;
    }
    ok &= team_barrier(ctr, (int)K * ++epoch);

    const int T = A.T;
    auto checked = [&](int t) { return t == T || (A.early_stop && t >= A.check_from); };
    int it = T, conv = 0;
    bool stopped = false;
    for (int t = 1; t <= T; ++t) {
        const bool vote = checked(t - 1);
        S.msg_in = mb[(t - 1) & 1];
        S.msg = mb[t & 1];
        const bool bad = res_check_phase<true, Msg, kGeneric>(c, S, d1[(t - 1) & 1], d1[t & 1], PK,
                                                              gw, NW);
        if (vote && wave_ballot(bad) != 0ull && lane == 0) flags[(size_t)t * A.F + f] = 1;
        ok &= team_barrier(ctr, (int)K * ++epoch);
        if (vote && agent_load(flags + (size_t)t * A.F + f) == 0) {
            // the decisions of iteration t - 1 satisfy H x = s: stop there
            it = t - 1;
            conv = 1;
            stopped = true;
            break;
        }
        res_group_sums<Msg>(c, S, part);
        __syncthreads();
        res_totals<Msg>(c, S, part);
        __syncthreads();
    }
    if (!stopped) {
        // the check of the last iteration (the channel decisions when T = 0)
        const bool bad = res_check_phase<false, Msg, kGeneric>(c, S, d1[T & 1], nullptr, PK, gw, NW);
        if (wave_ballot(bad) != 0ull && lane == 0) flags[(size_t)(T + 1) * A.F + f] = 1;
        ok &= team_barrier(ctr, (int)K * ++epoch);
        conv = agent_load(flags + (size_t)(T + 1) * A.F + f) == 0;
    }

    // Read-out over the frame's workgroups: decisions at the exit iteration
    // (every workgroup holds the same totals).
    const uint64_t *dexit = d1[it & 1];
    uint8_t *bits_out = A.bits_out + (size_t)f * c.n;
    for (unsigned v = gt; v < (unsigned)c.n; v += NT) {
        const unsigned col = v / Z, jj = v - col * Z;
        const int kind = c.col_kind[col];
        const unsigned ref = (unsigned)c.col_ref[col];
        int bit = llr[v] < 0.0f;
        if (kind == COL_CORE) {
            bit = tot[ref * Z + jj] < 0.0f;
        } else if (kind == COL_DEG1 && it > 0) {
            unsigned a = jj + Z - (unsigned)c.d1_shift[ref];
            a -= (a >= Z) ? Z : 0u;
            bit = (int)((dexit[ref * W + (a >> 6)] >> (a & 63u)) & 1ull);
        }
        bits_out[v] = (uint8_t)bit;
    }
    if (threadIdx.x == 0 && (k == 0 || !ok)) {
        A.iters_out[f] = ok ? it : -1;  // -1: a barrier wait ran out
        A.conv_out[f] = ok ? (uint8_t)conv : (uint8_t)0;
    }
}

__global__ void split_clear(int32_t *p, unsigned n) {
    const unsigned i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0;
}

}  // namespace

bool split_offered(const CodeDev &c, bool fp16) {
    return c.res_units > 0 && resident_layout(c, fp16).total <= kSplitMaxStateBytes;
}

// Workgroups per frame: up to kSplitMaxTeam while the frames' workgroups fit
// one per CU of the 256.
int split_team(int F) {
    const int slots = 8 * ((F + 7) / 8);
    int K = 256 / slots;
    return K < 1 ? 1 : (K > kSplitMaxTeam ? kSplitMaxTeam : K);
}

hipError_t enqueue_split(const DecodeLaunch &l, const WorkLayout &W) {
    const CodeDev &c = l.c;
    if (W.split_frame == 0) return hipErrorInvalidValue;
    const int K = split_team(l.F);
    SplitArgs a{};
    a.llr = l.llr;
    a.syndrome = l.syndrome;
    a.psi = reinterpret_cast<float *>(l.ws + W.psi);
    a.msg[0] = l.ws + W.msg;
    a.msg[1] = l.ws + W.split_msg;
    a.synbits = reinterpret_cast<uint64_t *>(l.ws + W.synbits);
    a.d1[0] = reinterpret_cast<uint64_t *>(l.ws + W.d1bits);
    a.d1[1] = a.d1[0] + (size_t)l.F * W.d1bits_frame;
    a.team = reinterpret_cast<int32_t *>(l.ws + W.team);
    a.bits_out = l.bits_out;
    a.iters_out = l.iters_out;
    a.conv_out = l.conv_out;
    a.msg_frame = W.split_frame;
    a.psi_frame = W.psi_frame;
    a.d1_frame = W.d1bits_frame;
    a.syn_frame = W.synbits_frame;
    a.T = l.T;
    a.early_stop = l.early_stop;
    a.check_from = l.check_from;
    a.K = K;
    a.F = l.F;
    const size_t nt = (size_t)c.NC * c.Z * 4;
    a.lds_q = (unsigned)nt;
    a.lds_part = (unsigned)(2 * nt);
    const size_t lds = (2 + kVnGroups) * nt;
    const unsigned nclear = (unsigned)((size_t)l.F * (l.T + 3));
    split_clear<<<dim3((nclear + 255) / 256), dim3(256), 0, l.stream>>>(a.team, nclear);
    const dim3 grid((unsigned)(8 * K * ((l.F + 7) / 8))), block(kSplitThreads);
    CodeDev cc = c;
    void *args[] = {&cc, &a};
    auto launch = [&](auto kernel) {
        hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void *>(kernel),
                                           hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess) return e;
        return hipLaunchCooperativeKernel(reinterpret_cast<const void *>(kernel), grid, block, args,
                                          (unsigned)lds, l.stream);
    };
    const bool generic = c.n_large > 0;
    if (l.fp16)
        return generic ? launch(split_decode<_Float16, true>) : launch(split_decode<_Float16, false>);
    return generic ? launch(split_decode<float, true>) : launch(split_decode<float, false>);
}

ResidentLayout resident_layout(const CodeDev &c, bool fp16) {
    auto a16 = [](size_t x) { return (x + 15) & ~(size_t)15; };
    ResidentLayout L{};
    L.tot = a16((size_t)c.NS * c.Z * (fp16 ? 2 : 4));
    L.q = a16(L.tot + (size_t)c.NC * c.Z * 4);
    L.part = a16(L.q + (size_t)c.NC * c.Z * 4);
    L.syn = a16(L.part + (size_t)kVnGroups * c.NC * c.Z * 4);
    L.d1 = L.syn + (size_t)c.mb * c.W * 8;
    L.flag = L.d1 + 2 * (size_t)c.ND1 * c.W * 8;
    L.total = a16(L.flag + 2 * 4);
    return L;
}

hipError_t enqueue_resident(const DecodeLaunch &l, const WorkLayout &W, size_t lds_limit) {
    const CodeDev &c = l.c;
    const ResidentLayout R = resident_layout(c, l.fp16 != 0);
    if (R.total > lds_limit) return hipErrorInvalidValue;
    ResidentArgs a{};
    a.llr = l.llr;
    a.syndrome = l.syndrome;
    a.psi = reinterpret_cast<float *>(l.ws + W.psi);
    a.bits_out = l.bits_out;
    a.iters_out = l.iters_out;
    a.conv_out = l.conv_out;
    a.psi_frame = W.psi_frame;
    a.T = l.T;
    a.early_stop = l.early_stop;
    a.check_from = l.check_from;
    a.lds_tot = (unsigned)R.tot;
    a.lds_q = (unsigned)R.q;
    a.lds_part = (unsigned)R.part;
    a.lds_syn = (unsigned)R.syn;
    a.lds_d1 = (unsigned)R.d1;
    a.lds_flag = (unsigned)R.flag;
    const dim3 grid((unsigned)l.F), block(kResThreads);
    auto launch = [&](auto kernel) {
        hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void *>(kernel),
                                           hipFuncAttributeMaxDynamicSharedMemorySize, (int)R.total);
        if (e != hipSuccess) return e;
        kernel<<<grid, block, R.total, l.stream>>>(c, a);
        return hipGetLastError();
    };
    const bool generic = c.n_large > 0;
    if (l.fp16)
        return generic ? launch(resident_decode<_Float16, true>)
                       : launch(resident_decode<_Float16, false>);
    return generic ? launch(resident_decode<float, true>) : launch(resident_decode<float, false>);
}

}  // namespace ldpc
