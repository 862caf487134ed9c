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
#include "passes.h"

#include <hip/hip_ext.h>

#include <algorithm>

namespace ldpc {

namespace {

using namespace dev;

// One launch covers the rows of one degree class; item i of the launch is
// (frame, row, tile) with the tile fastest, decoded with host-computed
// divisors.
template <typename Msg, bool kLarge, int MODE, int CPT>
__device__ __forceinline__ void check_pass_body(const CodeDev &c, const CnArgs &A, FastDiv tiles,
                                                FastDiv rows, unsigned frames) {
    const unsigned n = tiles.d * rows.d * frames;
    const unsigned i = xcd_item(blockIdx.x, n);
    if (i >= n) return;
    const unsigned i1 = fdiv(i, tiles);
    const unsigned tile = i - i1 * tiles.d;
    const unsigned f = fdiv(i1, rows);
    const int y = (kLarge ? c.n_small : 0) + (int)(i1 - f * rows.d);
    check_work<Msg, kLarge, MODE, CPT>(c, A, (int)f, y, tile);
}

template <typename Msg, int MODE, int CPT>
__global__ __launch_bounds__(kBlock) void check_pass(CodeDev c, CnArgs A, FastDiv tiles,
                                                     FastDiv rows, unsigned frames) {
    check_pass_body<Msg, false, MODE, CPT>(c, A, tiles, rows, frames);
}

// The check pass of a code with owner groups: per frame, the (row, tile)
// items of the common rows outside the t-domain class (row-list positions
// before and after its range) come first, then the (group, tile) items of the
// t-domain rows.  The former carry several times the work per check of the
// latter, so starting them first keeps them off the launch's tail.
template <typename Msg, int MODE, int CPT>
__global__ __launch_bounds__(kBlock) void check_pass_grouped(CodeDev c, CnArgs A, FastDiv per_frame,
                                                             FastDiv gtiles, FastDiv rtiles,
                                                             unsigned group_items,
                                                             unsigned frames) {
    const unsigned n = per_frame.d * frames;
    const unsigned i = xcd_item(blockIdx.x, n);
    if (i >= n) return;
    const unsigned f = fdiv(i, per_frame);
    const unsigned r0 = i - f * per_frame.d;
    const unsigned row_items = per_frame.d - group_items;
    // r: the item's position with the group items first, as decoded below
    const unsigned r = r0 < row_items ? r0 + group_items : r0 - row_items;
    if (r < group_items) {
        const unsigned g = fdiv(r, gtiles);
        group_work<MODE, Msg>(c, A, (int)f, (int)g, r - g * gtiles.d);
    } else {
        const unsigned r2 = r - group_items;
        const unsigned y0 = fdiv(r2, rtiles);
        const int lo = c.cls_end[kTdomClass - 1];
        const int y = (int)y0 < lo ? (int)y0 : (int)y0 + c.n_tdom;
        check_work<Msg, false, MODE, CPT>(c, A, (int)f, y, r2 - y0 * rtiles.d);
    }
}

template <typename Msg, int MODE, int CPT>
__global__ __launch_bounds__(kBlock) void check_pass_large(CodeDev c, CnArgs A, FastDiv tiles,
                                                           FastDiv rows, unsigned frames) {
    check_pass_body<Msg, true, MODE, CPT>(c, A, tiles, rows, frames);
}

// Common rows run with the requested checks per thread (1, 2 or 4); the rare
// generic rows, and launches that also write posteriors, with the default.
// A launch of 256-thread workgroups, optionally recording caller events at
// the start and end of the kernel's execution.
template <typename... KArgs, typename... Args>
void launch_timed(void (*kernel)(KArgs...), dim3 grid, hipStream_t st, hipEvent_t start,
                  hipEvent_t stop, Args... args) {
    if (start || stop)
        hipExtLaunchKernelGGL(kernel, grid, dim3(kBlock), 0, st, start, stop, 0, args...);
    else
        kernel<<<grid, dim3(kBlock), 0, st>>>(args...);
}

template <typename Msg, int MODE>
void launch_check_pass(const CodeDev &c, const CnArgs &a, int F, int cpt, hipStream_t st,
                       hipEvent_t start = nullptr, hipEvent_t stop = nullptr) {
    const bool both = c.n_small > 0 && c.n_large > 0;
    const unsigned fr = (unsigned)F;
    if constexpr (base_mode(MODE) != kVoteOnly) {
        if (c.n_groups > 0) {
            // owner groups (256 positions per item) and the other common rows
            if constexpr (with_post(MODE)) cpt = kDefaultChecksPerThread;
            const unsigned gt = (unsigned)((c.Z + kBlock - 1) / kBlock);
            const unsigned rt = check_tiles(c.Z, cpt);
            const unsigned gi = gt * (unsigned)c.n_groups;
            const unsigned per = gi + rt * (unsigned)(c.n_small - c.n_tdom);
            const dim3 g(xcd_grid(per * fr));
            const FastDiv dp = fast_div(per), dg = fast_div(gt), dr = fast_div(rt);
            hipEvent_t e1 = both ? nullptr : stop;
            if constexpr (with_post(MODE)) {
                launch_timed(check_pass_grouped<Msg, MODE, kDefaultChecksPerThread>, g, st, start,
                             e1, c, a, dp, dg, dr, gi, fr);
            } else {
                if (cpt == 1)
                    launch_timed(check_pass_grouped<Msg, MODE, 1>, g, st, start, e1, c, a, dp, dg,
                                 dr, gi, fr);
                else if (cpt == 2)
                    launch_timed(check_pass_grouped<Msg, MODE, 2>, g, st, start, e1, c, a, dp, dg,
                                 dr, gi, fr);
                else
                    launch_timed(check_pass_grouped<Msg, MODE, 4>, g, st, start, e1, c, a, dp, dg,
                                 dr, gi, fr);
            }
            if (c.n_large > 0) {
                const unsigned tl = check_tiles(c.Z, kDefaultChecksPerThread),
                               rows = (unsigned)c.n_large;
                launch_timed(check_pass_large<Msg, MODE, kDefaultChecksPerThread>,
                             dim3(xcd_grid(tl * rows * fr)), st, nullptr, stop, c, a,
                             fast_div(tl), fast_div(rows), fr);
            }
            return;
        }
    }
    if (c.n_small > 0) {
        if constexpr (with_post(MODE)) cpt = kDefaultChecksPerThread;
        const unsigned tl = check_tiles(c.Z, cpt), rows = (unsigned)c.n_small;
        const dim3 g(xcd_grid(tl * rows * fr));
        const FastDiv dt = fast_div(tl), dr = fast_div(rows);
        hipEvent_t e1 = both ? nullptr : stop;
        if constexpr (with_post(MODE)) {
            launch_timed(check_pass<Msg, MODE, kDefaultChecksPerThread>, g, st, start, e1, c, a,
                         dt, dr, fr);
        } else {
            if (cpt == 1)
                launch_timed(check_pass<Msg, MODE, 1>, g, st, start, e1, c, a, dt, dr, fr);
            else if (cpt == 2)
                launch_timed(check_pass<Msg, MODE, 2>, g, st, start, e1, c, a, dt, dr, fr);
            else
                launch_timed(check_pass<Msg, MODE, 4>, g, st, start, e1, c, a, dt, dr, fr);
        }
    }
    if (c.n_large > 0) {
        const unsigned tl = check_tiles(c.Z, kDefaultChecksPerThread), rows = (unsigned)c.n_large;
        launch_timed(check_pass_large<Msg, MODE, kDefaultChecksPerThread>,
                     dim3(xcd_grid(tl * rows * fr)), st, both ? nullptr : start, stop, c,
                     a, fast_div(tl), fast_div(rows), fr);
    }
}

template <int U, typename Msg>
__global__ __launch_bounds__(kBlock) void variable_pass(CodeDev c, VnArgs A, FastDiv tiles,
                                                        FastDiv cols, unsigned frames) {
    const unsigned n = tiles.d * cols.d * frames;
    const unsigned i = xcd_item(blockIdx.x, n);
    if (i >= n) return;
    const unsigned i1 = fdiv(i, tiles);
    const unsigned tile = i - i1 * tiles.d;
    const unsigned f = fdiv(i1, cols);
    if (A.fail[(size_t)(A.t - 1) * A.F + f] == 0) return;
    variable_work<U, Msg, vn_vpt<Msg>(), true>(c, A, (int)f, (int)(i1 - f * cols.d), tile);
}

template <typename Msg>
void launch_variable_pass(const CodeDev &c, const VnArgs &v, int F, hipStream_t st,
                          hipEvent_t start = nullptr, hipEvent_t stop = nullptr) {
    const unsigned tl = variable_tiles(c.Z, vn_vpt<Msg>());
    const dim3 g(xcd_grid(tl * (unsigned)c.NC * (unsigned)F));
    const FastDiv dt = fast_div(tl), dc = fast_div((unsigned)c.NC);
    const unsigned fr = (unsigned)F;
    switch (variable_group(2 * c.max_half_terms)) {
        case 4: launch_timed(variable_pass<4, Msg>, g, st, start, stop, c, v, dt, dc, fr); break;
        case 8: launch_timed(variable_pass<8, Msg>, g, st, start, stop, c, v, dt, dc, fr); break;
        case 13: launch_timed(variable_pass<13, Msg>, g, st, start, stop, c, v, dt, dc, fr); break;
        case 16: launch_timed(variable_pass<16, Msg>, g, st, start, stop, c, v, dt, dc, fr); break;
        default: launch_timed(variable_pass<26, Msg>, g, st, start, stop, c, v, dt, dc, fr); break;
    }
}

// fail[t][f] = 1 marks "iteration t not checked or check failed".
__global__ void init_fail(int32_t *fail, int F, int T, int early_stop, int check_from) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= (T + 1) * F) return;
    const int t = i / F;
    const bool checked = (t == T) || (early_stop && t >= check_from);
    fail[i] = checked ? 0 : 1;
}

__global__ __launch_bounds__(kBlock) void pack_syndrome(CodeDev c, const uint8_t *syn,
                                                        uint64_t *synbits, size_t syn_frame) {
    pack_syndrome_work(c, syn, synbits, syn_frame, blockIdx.z, blockIdx.y, blockIdx.x);
}

__global__ __launch_bounds__(kBlock) void init_totals(CodeDev c, const float *llr, float *tot,
                                                      size_t tot_frame) {
    init_totals_work(c, llr, tot, tot_frame, blockIdx.z, blockIdx.y, blockIdx.x);
}

__global__ __launch_bounds__(kBlock) void init_psi(CodeDev c, const float *llr, float *psi,
                                                   size_t psi_frame) {
    init_psi_work(c, llr, psi, psi_frame, blockIdx.z, blockIdx.y, blockIdx.x);
}

__global__ __launch_bounds__(64) void frame_exit(FinArgs A) { frame_exit_work(A, blockIdx.x); }

__global__ __launch_bounds__(kBlock) void finalize(CodeDev c, FinArgs A) {
    finalize_work(c, A, blockIdx.z, blockIdx.y, blockIdx.x);
}

__global__ __launch_bounds__(kBlock) void syndrome_kernel(CodeDev c, const uint8_t *bits,
                                                          uint8_t *syn) {
    const int f = blockIdx.z, r = blockIdx.y;
    const int a = blockIdx.x * kBlock + threadIdx.x;  // check index in the code as given
    if (a >= c.Z) return;
    const uint8_t *x = bits + (size_t)f * c.n;
    const int b0 = c.row_first[r], d = c.row_deg[r];
    int ar = a + c.row_rot[r];  // the same check in the relabelled tables
    ar -= (ar >= c.Z) ? c.Z : 0;
    int p = 0;
    for (int k = 0; k < d; ++k) {
        int j = ar + c.blk_shift[b0 + k];
        j -= (j >= c.Z) ? c.Z : 0;
        p ^= x[(size_t)c.blk_col[b0 + k] * c.Z + j] & 1;
    }
    syn[(size_t)f * c.m + (size_t)r * c.Z + a] = (uint8_t)p;
}

inline size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }
inline unsigned tiles(int n) { return (unsigned)((n + kBlock - 1) / kBlock); }

// The kernel sequence of one decode, in three parts so that two decodes can
// be interleaved launch by launch on two streams: set-up, one iteration
// (check pass and variable pass), and the final vote and read-out.
template <typename Msg>
struct Sequence {
    const DecodeLaunch &l;
    WorkLayout L;
    CnArgs a{};
    VnArgs v{};
    uint64_t *d1b[2];
    float *d1p[2] = {nullptr, nullptr};
    int32_t *fail;
    float *tot, *psi;
    uint64_t *synbits;

    Sequence(const DecodeLaunch &launch, const WorkLayout &layout) : l(launch), L(layout) {
        const int F = l.F;
        char *ws = l.ws;
        tot = reinterpret_cast<float *>(ws + L.tot);
        psi = reinterpret_cast<float *>(ws + L.psi);
        synbits = reinterpret_cast<uint64_t *>(ws + L.synbits);
        d1b[0] = reinterpret_cast<uint64_t *>(ws + L.d1bits);
        d1b[1] = d1b[0] + (size_t)F * L.d1bits_frame;
        fail = reinterpret_cast<int32_t *>(ws + L.fail);
        if (l.llr_out) {
            d1p[0] = reinterpret_cast<float *>(ws + L.d1post);
            d1p[1] = d1p[0] + (size_t)F * L.psi_frame;
        }
        a.llr = l.llr;
        a.psi = psi;
        a.msg = ws + L.msg;
        a.tot = tot;
        a.synbits = synbits;
        a.fail = fail;
        a.msg_frame = L.msg_frame;
        a.tot_frame = L.tot_frame;
        a.d1_frame = L.d1bits_frame;
        a.syn_frame = L.synbits_frame;
        a.psi_frame = L.psi_frame;
        a.part = reinterpret_cast<float *>(ws + L.part);
        a.part_frame = L.part_frame;
        a.F = F;
        v.llr = l.llr;
        v.msg = a.msg;
        v.tot = tot;
        v.fail = fail;
        v.msg_frame = L.msg_frame;
        v.tot_frame = L.tot_frame;
        v.part = a.part;
        v.part_frame = L.part_frame;
        v.F = F;
    }

    bool checked(int t) const { return t == l.T || (l.early_stop && t >= l.check_from); }

    void setup() {
        const CodeDev &c = l.c;
        const int F = l.F;
        hipStream_t st = l.stream;
        const int nfail = (l.T + 1) * F;
        init_fail<<<dim3((nfail + kBlock - 1) / kBlock), dim3(kBlock), 0, st>>>(fail, F, l.T,
                                                                               l.early_stop,
                                                                               l.check_from);
        pack_syndrome<<<dim3(setup_tiles(c.Z), c.mb, F), dim3(kBlock), 0, st>>>(c, l.syndrome, synbits,
                                                                         L.synbits_frame);
        if (c.NC > 0)
            init_totals<<<dim3(setup_tiles(c.Z), c.NC, F), dim3(kBlock), 0, st>>>(c, l.llr, tot,
                                                                           L.tot_frame);
        if (c.ND1 > 0)
            init_psi<<<dim3(setup_tiles(c.Z), c.ND1, F), dim3(kBlock), 0, st>>>(c, l.llr, psi,
                                                                         L.psi_frame);
    }

    void iteration(int t) {
        const CodeDev &c = l.c;
        hipStream_t st = l.stream;
        a.t = t;
        a.vote = checked(t - 1) ? 1 : 0;
        a.d1_from_llr = (t == 1);
        a.d1_prev = d1b[(t - 1) & 1];
        a.d1_cur = d1b[t & 1];
        a.d1post = d1p[t & 1];
        a.skip_after = t >= 2 ? t - 2 : -1;
        hipEvent_t *ev = l.events ? l.events + 4 * (t - 1) : nullptr;
        hipEvent_t e0 = ev ? ev[0] : nullptr, e1 = ev ? ev[1] : nullptr;
        if (t == 1) {
            if (a.d1post)
                launch_check_pass<Msg, kFirst | kPost>(c, a, l.F, l.cpt, st, e0, e1);
            else
                launch_check_pass<Msg, kFirst>(c, a, l.F, l.cpt, st, e0, e1);
        } else {
            if (a.d1post)
                launch_check_pass<Msg, kSteady | kPost>(c, a, l.F, l.cpt, st, e0, e1);
            else
                launch_check_pass<Msg, kSteady>(c, a, l.F, l.cpt, st, e0, e1);
        }
        if (c.NC > 0) {
            v.t = t;
            launch_variable_pass<Msg>(c, v, l.F, st, ev ? ev[2] : nullptr, ev ? ev[3] : nullptr);
        } else if (ev) {
            (void)hipEventRecord(ev[2], st);
            (void)hipEventRecord(ev[3], st);
        }
    }

    void finish() {
        const CodeDev &c = l.c;
        const int F = l.F, T = l.T;
        hipStream_t st = l.stream;
        // the check of the last iteration (or of the channel decisions when T = 0)
        a.t = T;
        a.vote = 1;
        a.d1_from_llr = (T == 0);
        a.d1_prev = d1b[T & 1];
        a.d1_cur = nullptr;
        a.d1post = nullptr;
        a.skip_after = T >= 1 ? T - 1 : -1;
        launch_check_pass<Msg, kVoteOnly>(c, a, F, l.cpt, st);

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
        frame_exit<<<dim3(F), dim3(64), 0, st>>>(fa);
        finalize<<<dim3(tiles(c.Z), c.nb, F), dim3(kBlock), 0, st>>>(c, fa);
    }
};

// One decode on one stream, or the two halves of the frames on the caller's
// stream and the library's second stream, launch by launch in turn, so that
// each half's kernels fill the other's gaps between dependent passes.
template <typename Msg>
hipError_t enqueue_typed(const DecodeLaunch &l, const WorkLayout &L) {
    Sequence<Msg> s(l, L);
    s.setup();
    for (int t = 1; t <= l.T; ++t) s.iteration(t);
    s.finish();
    return hipGetLastError();
}

template <typename Msg>
hipError_t enqueue_pair(const DecodeLaunch &la, const WorkLayout &La, const DecodeLaunch &lb,
                        const WorkLayout &Lb) {
    Sequence<Msg> sa(la, La), sb(lb, Lb);
    sa.setup();
    sb.setup();
    for (int t = 1; t <= la.T; ++t) {
        sa.iteration(t);
        sb.iteration(t);
    }
    sa.finish();
    sb.finish();
    return hipGetLastError();
}

}  // namespace

WorkLayout work_layout(const CodeDev &c, int F, int T, bool fp16, bool want_llr) {
    WorkLayout L{};
    L.msg_frame = (size_t)c.NS * c.Zp;
    L.tot_frame = (size_t)c.NC * c.Zt;
    L.d1bits_frame = (size_t)c.ND1 * c.W;
    L.synbits_frame = (size_t)c.mb * c.W;
    L.psi_frame = (size_t)c.ND1 * c.Zp;
    size_t off = 0;
    L.msg = off;
    off = align256(off + ((size_t)F * L.msg_frame + kLanePad) * (fp16 ? 2 : 4));
    L.tot = off;
    off = align256(off + (size_t)F * L.tot_frame * 4);
    L.psi = off;
    off = align256(off + ((size_t)F * L.psi_frame + kLanePad) * 4);
    L.d1bits = off;
    off = align256(off + 2 * (size_t)F * L.d1bits_frame * 8);
    L.synbits = off;
    off = align256(off + (size_t)F * L.synbits_frame * 8);
    L.fail = off;
    off = align256(off + (size_t)(T + 1) * F * 4);
    L.d1post = off;
    if (want_llr) off = align256(off + 2 * (size_t)F * L.psi_frame * 4);
    L.part_frame = (size_t)c.n_groups * c.Zp;
    L.part = off;
    off = align256(off + (size_t)F * L.part_frame * 4);
    L.split_frame = split_offered(c, fp16) ? (size_t)c.NS * c.Z : 0;
    L.split_msg = off;
    off = align256(off + (size_t)F * L.split_frame * (fp16 ? 2 : 4));
    // frame-split schedule: F arrival counters, then (T + 2) * F vote flags
    L.team = off;
    off = align256(off + (size_t)F * (T + 3) * 4);
    L.total = off;
    return L;
}

// Frames of the first half when a decode runs on two streams.
static int first_half(int F) { return (F + 1) / 2; }

size_t decode_workspace_bytes(const CodeDev &c, int F, int T, bool fp16, bool want_llr) {
    const size_t one = work_layout(c, F, T, fp16, want_llr).total;
    if (F < 2) return one;
    const int F1 = first_half(F);
    const size_t two = work_layout(c, F1, T, fp16, want_llr).total +
                       work_layout(c, F - F1, T, fp16, want_llr).total;
    return std::max(one, two);
}

hipError_t enqueue_decode(const DecodeLaunch &l) {
    if (l.F >= 2 && !l.events && l.aux && l.fork && l.join) {
        const bool fp16 = l.fp16 != 0, llr = l.llr_out != nullptr;
        const int F1 = first_half(l.F);
        DecodeLaunch a = l, b = l;
        a.F = F1;
        b.F = l.F - F1;
        const WorkLayout La = work_layout(l.c, a.F, l.T, fp16, llr);
        const WorkLayout Lb = work_layout(l.c, b.F, l.T, fp16, llr);
        b.llr = l.llr + (size_t)F1 * l.c.n;
        b.syndrome = l.syndrome + (size_t)F1 * l.c.m;
        b.bits_out = l.bits_out + (size_t)F1 * l.c.n;
        b.iters_out = l.iters_out + F1;
        b.conv_out = l.conv_out + F1;
        b.llr_out = l.llr_out ? l.llr_out + (size_t)F1 * l.c.n : nullptr;
        b.ws = l.ws + La.total;
        b.stream = l.aux;
        hipError_t e = hipEventRecord(l.fork, l.stream);
        if (e == hipSuccess) e = hipStreamWaitEvent(l.aux, l.fork, 0);
        if (e != hipSuccess) return e;
        e = fp16 ? enqueue_pair<_Float16>(a, La, b, Lb) : enqueue_pair<float>(a, La, b, Lb);
        if (e == hipSuccess) e = hipEventRecord(l.join, l.aux);
        if (e == hipSuccess) e = hipStreamWaitEvent(l.stream, l.join, 0);
        return e;
    }
    const WorkLayout L = work_layout(l.c, l.F, l.T, l.fp16 != 0, l.llr_out != nullptr);
    return l.fp16 ? enqueue_typed<_Float16>(l, L) : enqueue_typed<float>(l, L);
}

hipError_t enqueue_syndrome(const CodeDev &c, int F, const uint8_t *bits, uint8_t *syn,
                            hipStream_t stream) {
    syndrome_kernel<<<dim3(tiles(c.Z), c.mb, F), dim3(kBlock), 0, stream>>>(c, bits, syn);
    return hipGetLastError();
}

}  // namespace ldpc
