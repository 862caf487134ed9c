// Internal declarations shared by the decoder kernels (decoder.hip) and the
// C-ABI layer (api.hip).  Not part of the public interface.
#pragma once

#include <hip/hip_runtime.h>

#include "../../include/ldpc.h"

#include <cstddef>
#include <cstdint>

namespace ldpc {

// Kinds of a non-zero base block, decided by the degree of its base column.
//  STATE: the column has degree >= 2, so the block's Z check-to-variable
//         messages are kept between iterations (the "state" edges).
//  DEG1:  the column has degree 1.  Its variable-to-check message is the
//         constant channel LLR (no other check feeds it), so nothing is stored;
//         the posterior is Q + m and is formed only for decisions (the long
//         diagonal of degree-1 parity bits, Sec. III-C).
enum : int32_t { KIND_STATE = 0, KIND_DEG1 = 1 };
enum : int32_t { COL_CORE = 0, COL_DEG1 = 1, COL_DEG0 = 2 };

// Check rows up to this degree with at most one degree-1 block share one
// kernel; every other row (up to LDPC_MAX_ROW_DEGREE) goes to a generic one,
// so their register needs do not lower the occupancy of the common rows.
constexpr int kSmallRowDegree = 6;

// Common rows come in 2 * kSmallRowDegree classes (degree D, stored blocks
// D - 1 or D); class index 2 (D - 1) + (stored - (D - 1)).
constexpr int kFixedClasses = 2 * kSmallRowDegree;
// The common-row class (degree 3, 2 stored blocks) whose check update runs in
// the t-domain (see tdom_check3).
constexpr int kTdomClass = 4;
// Words of a common row's descriptor (see CodeDev::row_desc).
constexpr int kRowDescWords = 20;

// Owner groups.  Every row of the t-domain class has two core blocks; one of
// them, chosen so that the core columns own about equally many rows, is the
// row's owner block.  The row's checks are relabelled (check a becomes
// (a + s) mod Z, s the owner block's shift), so the owner block has shift 0
// and the row's check a meets the owner column at position a.  Rows with the
// same owner column, kGroupRows at a time in increasing row order, form a
// group; a group's checks at one position all feed the same core variable,
// so the check pass adds their messages to that variable into one partial
// sum per group, and the variable pass reads the partial instead of the
// group's messages.
// Measured on the rate-0.02 template (24 owned rows per core column) at
// Z = 6667, 8 frames decoded as two halves on two streams: groups of 12 rows
// 2374 Mbit/s, against 2333 (16), 2231 (24) and 2245 (8); with half messages
// 3130 against 2981, 2850 and 2727.  Twice as many group items as with 24
// outweigh the extra partials the variable pass reads (with one stream per
// decode, 24 had measured fastest).
constexpr int kGroupRows = 12;
constexpr int kGroupDescWords = 8;

// Words of a row's descriptor for the frame-resident schedule (see
// CodeDev::res_desc), and the blocks its variable phase reads per batch.
constexpr int kResDescWords = 24;
constexpr int kResVnBatch = 16;

// Default and largest checks per thread of the common-row check kernel.
constexpr int kDefaultChecksPerThread = 4;
constexpr int kMaxChecksPerThread = 4;

// Elements read past the end of a per-block array by the padding lanes of the
// last check tile of a row (256 threads x 4 checks); the message and degree-1
// regions carry this much slack.
constexpr int kLanePad = 256 * kMaxChecksPerThread;

// Device view of a code: sizes plus pointers into small device tables.  Passed
// by value as a kernel argument; every table index below is uniform across a
// workgroup, so the loads are scalar.
struct CodeDev {
    int32_t Z, mb, nb, n, m;
    int32_t NS;   // state blocks (messages per frame = NS * Zp)
    int32_t NC;   // core columns (degree >= 2)
    int32_t ND1;  // degree-1 columns (= degree-1 blocks)
    int32_t W;    // 64-bit words per Z bits
    // Row stride of the core totals: row k holds L[j] at j and again at j + Z,
    // so a check gathers position (a + s) mod Z as index a + s without a wrap;
    // kLanePad more slots keep padding lanes in bounds.
    int32_t Zt;
    // Stride of the per-block arrays (messages, Psi, degree-1 posteriors): Z
    // rounded up to 64, so every block starts on a 256-byte boundary.
    int32_t Zp;
    // per base row r: blocks row_first[r] .. row_first[r] + row_deg[r] - 1;
    // the first row_ns[r] are blocks of columns of degree >= 2 (stored
    // messages), the rest degree-1 blocks, each group in column order
    const int32_t *row_first, *row_deg, *row_ns;
    // base rows ordered by class: the n_small common rows (degree
    // <= kSmallRowDegree, at most one degree-1 block) first, then the n_large others
    const int32_t *row_list;
    int32_t n_small, n_large;
    // the common rows are grouped by class in row_list: class i holds positions
    // cls_end[i-1] .. cls_end[i] - 1 (cls_end[-1] = 0)
    int32_t cls_end[kFixedClasses];
    // per common row (row_list position y), kRowDescWords words at y * kRowDescWords:
    //   [0, 6)  stored block k: offset of its column's totals + shift (core * Zt + s)
    //   [6, 12) stored block k: offset of its messages (state index * Zp)
    //   12..15  degree-1 block: Psi offset (index * Zp), decision-word offset
    //           (index * W), channel-LLR offset (column * Z), shift
    //   16, 17  syndrome-word offset (r * W), base row r
    //   18      the row's class
    const int32_t *row_desc;
    // per block: shift, kind, ref (state index or degree-1 index), column,
    // core index of the column (state blocks only, else -1)
    const int32_t *blk_shift, *blk_kind, *blk_ref, *blk_col, *blk_core;
    // per core column k: its base column, and its state blocks
    // core_state[core_first[k] + i], core_shift[...], i < core_deg[k], in
    // increasing row order
    const int32_t *core_col, *core_first, *core_deg, *core_state, *core_shift;
    // the same blocks as (message offset state * Zp, shift) pairs, column k at
    // core_tab[k * core_tab_stride], so a column's entries are addressed
    // without loading core_first first
    const int32_t *core_tab;
    int32_t core_tab_stride;
    // frame-resident schedule (offsets into a frame's LDS arrays, Z per block):
    // per base row r, kResDescWords words at r * kResDescWords:
    //   0 class (0..11 common classes as above, 12 / 13 other rows of degree
    //     <= 8 / <= 16), 1 degree, 2 stored blocks, 3 first block, 4 r * W
    //   [5, 11)  common rows, block k: stored: core * Z (totals), degree-1:
    //            index * Zp (Psi)
    //   [11, 17) stored: state index * Z (messages), degree-1: index * W
    //            (decision words)
    //   [17, 23) shift of block k
    // and per core column k, at res_core[k * res_core_stride], its blocks as
    // (state index * Z, shift) pairs in increasing row order (rows padded with
    // zero pairs to a multiple of kResVnBatch pairs, and kResVnBatch more
    // pairs after the last)
    const int32_t *res_desc, *res_core;
    int32_t res_core_stride;
    // the check-phase units (base row r, chunk ch of 64 checks) as r | ch << 16,
    // rows in class order; res_units = mb * W, or 0 where the schedule is not
    // offered (a table that large would never fit LDS)
    const int32_t *res_unit;
    int32_t res_units;
    int32_t max_core_deg;  // largest degree of a core column
    // per base column: kind and index within its kind
    const int32_t *col_kind, *col_ref;
    // per degree-1 column: its base column and the shift of its only block
    const int32_t *d1_col, *d1_shift;
    // per degree-1 column: 1 if its row is of class (degree 3, 2 stored
    // blocks), updated in the t-domain, so its input is +-e^{-|Q|} rather than
    // +-Phi(|Q|)
    const int32_t *d1_tdom;
    // per base row r: the relabelling of its checks: check a of the code as
    // given is check (a + row_rot[r]) mod Z of the tables above (0 for rows
    // without an owner)
    const int32_t *row_rot;
    // owner groups: per group g, grp_hdr[4 g ..] = owner column's totals
    // offset (core * Zt), row count, 0, 0; per row i of the group,
    // kGroupDescWords words at grp_desc[(g kGroupRows + i) kGroupDescWords]:
    //   0 owner block's message offset (state index * Zp), 1 the other core
    //   block's message offset, 2 the other block's totals offset plus shift
    //   (core * Zt + s), 3 Psi offset (degree-1 index * Zp), 4 decision-word
    //   offset (degree-1 index * W), 5 syndrome-word offset (r * W),
    //   6 degree-1 column's LLR offset (column * Z), 7 degree-1 shift
    int32_t n_groups, n_tdom;  // groups; rows of the t-domain class
    const int32_t *grp_hdr, *grp_desc;
    // per core column k: the first core_own[k] entries of core_tab and
    // res_core are its owned blocks, group by group (kGroupRows per group,
    // rows increasing), the rest its other blocks (rows increasing);
    // core_ngrp[k] groups, numbered from core_grp0[k].  The column's total is
    //   L = (Q log2(e) + S0) + S1,
    // over the terms P_0 .. P_{G-1} (group partials, each summed from +0 in
    // row order) followed by the other blocks' messages: S0 sums the first
    // ceil(terms / 2) terms from +0, S1 the rest.
    const int32_t *core_own, *core_ngrp, *core_grp0;
    int32_t max_half_terms;  // largest ceil(terms / 2) over the core columns
};

// Byte offsets of the decode workspace for F frames and T iterations.
struct WorkLayout {
    size_t msg, tot, psi, d1bits, synbits, fail, d1post, part, split_msg, team, total;
    size_t part_frame;     // floats per frame (group partials, n_groups * Zp)
    size_t split_frame;    // messages per frame of the frame-split schedule's second
                           // buffer (NS * Z, or 0 where that schedule is not offered)
    size_t msg_frame;      // elements per frame
    size_t tot_frame;      // floats per frame
    size_t psi_frame;      // floats per frame (degree-1 inputs; also posteriors)
    size_t d1bits_frame;   // words per frame
    size_t synbits_frame;  // words per frame
};

WorkLayout work_layout(const CodeDev &c, int F, int T, bool fp16, bool want_llr);

struct DecodeLaunch {
    CodeDev c;
    int F, T;
    int early_stop, check_from, fp16;
    int cpt;               // checks per thread of the common-row check kernel (1, 2, 4)
    const float *llr;
    const uint8_t *syndrome;
    uint8_t *bits_out;
    int32_t *iters_out;
    uint8_t *conv_out;
    float *llr_out;
    char *ws;
    hipEvent_t *events;    // optional: 4T caller events, start and end of each iteration kernel
    hipStream_t stream;
    // the library's second stream and its fork / join events: the per-iteration
    // launches of F >= 2 frames (without caller events) run the two halves of the
    // frames on `stream` and `aux`, joined back into `stream` (null: one stream)
    hipStream_t aux;
    hipEvent_t fork, join;
};

// Enqueue the whole decode on l.stream.  Returns hipSuccess or the first
// launch error.
hipError_t enqueue_decode(const DecodeLaunch &l);
// Workspace bytes of a decode on any schedule (the two-stream split of the
// launches takes two independent layouts of half the frames each).
size_t decode_workspace_bytes(const CodeDev &c, int F, int T, bool fp16, bool want_llr);

// Frame-resident schedule (resident.hip): one workgroup per frame runs every
// iteration with the frame's state in LDS.  Byte offsets of that state:
struct ResidentLayout {
    size_t tot, q, part, syn, d1, flag, total;  // messages at 0; total = LDS bytes per workgroup
};
ResidentLayout resident_layout(const CodeDev &c, bool fp16);

struct ResidentArgs {
    const float *llr;          // [F][n]
    const uint8_t *syndrome;   // [F][m]
    float *psi;                // [F][ND1][Zp] degree-1 inputs (decode workspace)
    uint8_t *bits_out;
    int32_t *iters_out;
    uint8_t *conv_out;
    size_t psi_frame;
    int T, early_stop, check_from;
    unsigned lds_tot, lds_q, lds_part, lds_syn, lds_d1, lds_flag;
};

// Enqueue a whole decode as one resident launch (no posteriors, no per-pass
// events).  hipErrorInvalidValue if the state exceeds lds_limit bytes.
hipError_t enqueue_resident(const DecodeLaunch &l, const WorkLayout &W, size_t lds_limit);

// Frame-split schedule (resident.hip): K co-resident workgroups per frame run
// every iteration in one cooperative launch, the frame's messages in global
// memory (two buffers, by iteration parity), the core totals in every
// workgroup's LDS, one barrier across the frame's workgroups per iteration.
// Offered where the frame's state is at most kSplitMaxStateBytes.
constexpr size_t kSplitMaxStateBytes = 160 * 1024;
constexpr int kSplitMaxTeam = 4;
constexpr int kSplitMaxFrames = 256;  // one 1024-thread workgroup per CU at most
bool split_offered(const CodeDev &c, bool fp16);
int split_team(int F);  // workgroups per frame for F frames
hipError_t enqueue_split(const DecodeLaunch &l, const WorkLayout &W);
hipError_t enqueue_syndrome(const CodeDev &c, int F, const uint8_t *bits, uint8_t *syn,
                            hipStream_t stream);
hipError_t enqueue_reconciliation_llr(int d, int F, int n, const float *x, const float *m,
                                      float sigma2, float *llr, hipStream_t stream);
hipError_t enqueue_reconciliation_message(int d, int F, int n, const uint8_t *bits, const float *y,
                                          float *m, hipStream_t stream);

}  // namespace ldpc
