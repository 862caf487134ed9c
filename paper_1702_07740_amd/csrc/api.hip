// C ABI of libldpc.so (declared in include/ldpc.h): argument checking, code
// tables, workspace sizing, and the enqueue of the decoder kernels.
#include "../../include/ldpc.h"
#include "engine.h"
#include "internal.h"

#include <cstdarg>
#include <cstdio>
#include <mutex>
#include <new>
#include <cstring>
#include <string>
#include <algorithm>
#include <vector>

using ldpc::CodeDev;

struct ldpc_code {
    ldpc_code_info_t info;
    int device;
    size_t lds_limit;       // LDS bytes one workgroup may take on that device
    CodeDev dev;            // sizes + device table pointers
    int32_t *table;         // one device allocation holding every table
    // the second stream of two-stream decodes, its fork and join events, and
    // the lock that keeps one call's record / wait pairs together (it also
    // guards the decode graphs below)
    hipStream_t aux = nullptr;
    hipEvent_t fork = nullptr, join = nullptr;
    std::mutex aux_lock;
    // Decode graphs.  A small one-stream decode on the per-iteration launches
    // that repeats an earlier call's sizes, options and pointers is captured
    // into a HIP graph (on `cap`, a stream of its own) at its second call and
    // replayed from the third, which saves the host two launches per
    // iteration.  kGraphSlots
    // entries, the least recently used one replaced (its count starts again).
    static constexpr int kGraphSlots = 4;
    static constexpr int kGraphKeyWords = 16;
    struct GraphSlot {
        int64_t key[kGraphKeyWords] = {};
        int seen = 0;                  // calls with this key; -1: capture failed
        hipGraphExec_t exec = nullptr;
        uint64_t used = 0;
    };
    hipStream_t cap = nullptr;
    GraphSlot graphs[kGraphSlots];
    uint64_t graph_clock = 0;
};

namespace {

thread_local std::string g_last_error;

int fail_with(int status, const char *fmt, ...) __attribute__((format(printf, 2, 3)));
int fail_with(int status, const char *fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_last_error = buf;
    return status;
}

// Decode workspace of ldpc_decode_batch_noalloc: one fixed region per device,
// part of this library's device code (the loader places it with the code and
// it stays until the process ends).  In host code the name `scratch` is only a
// host-side stand-in; the region's device address on each device comes from
// hipGetSymbolAddress, looked up once per device with that device current.
constexpr size_t kScratchBytes = LDPC_NOALLOC_SCRATCH_BYTES;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_lock;
void *g_scratch_ptr[kMaxDevices] = {};

// Look up (once) the scratch region's address on `device`, which must be
// the current device.
hipError_t scratch_setup(int device) {
    if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> guard(g_scratch_lock);
    if (g_scratch_ptr[device]) return hipSuccess;
    void *p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    if (!p || (reinterpret_cast<uintptr_t>(p) & 255)) return hipErrorInvalidSymbol;
    g_scratch_ptr[device] = p;
    return hipSuccess;
}

void *scratch_ptr(int device) {
    if (device < 0 || device >= kMaxDevices) return nullptr;
    std::lock_guard<std::mutex> guard(g_scratch_lock);
    return g_scratch_ptr[device];
}

int check_device(const ldpc_code *code) {
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return fail_with(LDPC_EDEVICE, "hipGetDevice: %s", hipGetErrorString(e));
    if (dev != code->device)
        return fail_with(LDPC_EDEVICE, "current device %d is not the code's device %d", dev,
                         code->device);
    return LDPC_OK;
}

}  // namespace

extern "C" {

const char *ldpc_status_string(int status) {
    switch (status) {
        case LDPC_OK: return "ok";
        case LDPC_EINVAL: return "invalid argument";
        case LDPC_ENOMEM: return "out of memory";
        case LDPC_EDEVICE: return "HIP device error";
        case LDPC_EUNSUPPORTED: return "unsupported code";
        case LDPC_EWORKSPACE: return "workspace missing, too small or misaligned";
        default: return "unknown status";
    }
}

const char *ldpc_last_error(void) { return g_last_error.c_str(); }

void ldpc_decode_opts_init(ldpc_decode_opts *o) {
    if (!o) return;
    o->early_stop = 1;
    o->check_from_iter = 0;
    o->msg_fp16 = 0;
    o->checks_per_thread = 0;
    o->llr_out = nullptr;
    o->timing_events = nullptr;
    o->n_timing_events = 0;
    o->schedule = LDPC_SCHEDULE_AUTO;
    o->streams = 0;
    o->graphs = 0;
}

int ldpc_code_create(int32_t mb, int32_t nb, const int32_t *base, int32_t Z, ldpc_code **out) {
    if (!out) return fail_with(LDPC_EINVAL, "out is null");
    *out = nullptr;
    if (!base) return fail_with(LDPC_EINVAL, "base is null");
    if (mb < 1 || nb < 1 || Z < 1) return fail_with(LDPC_EINVAL, "mb, nb, Z must be >= 1");
    if ((int64_t)nb * Z >= (1ll << 31) || (int64_t)mb * Z >= (1ll << 31))
        return fail_with(LDPC_EINVAL, "code too long: nb*Z and mb*Z must be < 2^31");

    // column degrees and classes
    std::vector<int32_t> col_deg(nb, 0);
    for (int r = 0; r < mb; ++r)
        for (int c = 0; c < nb; ++c) {
            const int32_t s = base[(size_t)r * nb + c];
            if (s < -1 || s >= Z)
                return fail_with(LDPC_EINVAL, "base[%d][%d] = %d is outside [-1, Z)", r, c, s);
            if (s >= 0) col_deg[c]++;
        }
    std::vector<int32_t> col_kind(nb), col_ref(nb);
    std::vector<int32_t> core_col, d1_col;
    for (int c = 0; c < nb; ++c) {
        if (col_deg[c] >= 2) {
            col_kind[c] = ldpc::COL_CORE;
            col_ref[c] = (int32_t)core_col.size();
            core_col.push_back(c);
        } else if (col_deg[c] == 1) {
            col_kind[c] = ldpc::COL_DEG1;
            col_ref[c] = (int32_t)d1_col.size();
            d1_col.push_back(c);
        } else {
            col_kind[c] = ldpc::COL_DEG0;
            col_ref[c] = -1;
        }
    }
    // Owner of each row of the t-domain class (two core blocks and one
    // degree-1 block): of its two core columns, the one that owns fewer rows
    // so far (ties: the lower column).  The row's checks are relabelled so
    // the owner block gets shift 0: every shift of the row drops by the owner
    // block's shift (mod Z).
    std::vector<int32_t> row_rot(mb, 0), row_owner(mb, -1);
    {
        std::vector<int32_t> owned(nb, 0);
        for (int r = 0; r < mb; ++r) {
            int ncore = 0, nd1 = 0, cc[2] = {-1, -1};
            for (int c = 0; c < nb; ++c) {
                if (base[(size_t)r * nb + c] < 0) continue;
                if (col_kind[c] == ldpc::COL_CORE) {
                    if (ncore < 2) cc[ncore] = c;
                    ++ncore;
                } else {
                    ++nd1;
                }
            }
            if (ncore != 2 || nd1 != 1) continue;
            const int o = owned[cc[1]] < owned[cc[0]] ? cc[1] : cc[0];
            owned[o]++;
            row_owner[r] = o;
            row_rot[r] = base[(size_t)r * nb + o];
        }
    }
    auto shift_of = [&](int r, int c) {
        const int32_t s = base[(size_t)r * nb + c] - row_rot[r];
        return s < 0 ? s + Z : s;
    };
    // blocks in row-major order; state blocks numbered in that order
    std::vector<int32_t> row_first(mb), row_deg(mb);
    std::vector<int32_t> blk_shift, blk_kind, blk_ref, blk_col, blk_core;
    std::vector<int32_t> d1_shift(d1_col.size(), 0), d1_row(d1_col.size(), 0);
    std::vector<int32_t> st_row, st_core, st_shift;
    int maxdeg = 0;
    std::vector<int32_t> row_ns(mb);
    for (int r = 0; r < mb; ++r) {
        row_first[r] = (int32_t)blk_shift.size();
        int d = 0;
        // within a row: blocks of stored columns first (the owner block
        // leading), then degree-1 blocks, each group in increasing column order
        std::vector<int> cols;
        if (row_owner[r] >= 0) cols.push_back(row_owner[r]);
        for (int c = 0; c < nb; ++c)
            if (base[(size_t)r * nb + c] >= 0 && col_kind[c] == ldpc::COL_CORE && c != row_owner[r])
                cols.push_back(c);
        row_ns[r] = (int32_t)cols.size();
        for (int c = 0; c < nb; ++c)
            if (base[(size_t)r * nb + c] >= 0 && col_kind[c] != ldpc::COL_CORE) cols.push_back(c);
        for (int c : cols) {
            const int32_t s = shift_of(r, c);
            ++d;
            blk_shift.push_back(s);
            blk_col.push_back(c);
            if (col_kind[c] == ldpc::COL_CORE) {
                blk_kind.push_back(ldpc::KIND_STATE);
                blk_ref.push_back((int32_t)st_row.size());
                blk_core.push_back(col_ref[c]);
                st_row.push_back(r);
                st_core.push_back(col_ref[c]);
                st_shift.push_back(s);
            } else {
                blk_kind.push_back(ldpc::KIND_DEG1);
                blk_ref.push_back(col_ref[c]);
                blk_core.push_back(-1);
                d1_shift[col_ref[c]] = s;
                d1_row[col_ref[c]] = r;
            }
        }
        row_deg[r] = d;
        if (d == 0) return fail_with(LDPC_EUNSUPPORTED, "base row %d has no block", r);
        if (d > LDPC_MAX_ROW_DEGREE)
            return fail_with(LDPC_EUNSUPPORTED, "base row %d has degree %d > %d", r, d,
                             LDPC_MAX_ROW_DEGREE);
        if (d > maxdeg) maxdeg = d;
    }
    const int NS = (int)st_row.size(), NC = (int)core_col.size(), ND1 = (int)d1_col.size();
    if (mb > 65535 || nb > 65535)  // base rows and base columns index grid.y
        return fail_with(LDPC_EUNSUPPORTED, "more than 65535 base rows or base columns");
    {
        // every per-frame array is addressed with 32-bit byte offsets
        const int64_t lim = (1ll << 30) - ldpc::kLanePad;
        const int64_t zt = ((2ll * Z + ldpc::kLanePad) + 63) / 64 * 64;
        const int64_t zp = ((int64_t)Z + 63) / 64 * 64;
        if ((int64_t)nb * Z >= lim || (int64_t)mb * Z >= lim || (int64_t)NS * zp >= lim ||
            (int64_t)ND1 * zp >= lim || (int64_t)NC * zt >= lim)
            return fail_with(LDPC_EINVAL,
                             "code too large: n, m, stored edges and 2 x core variables per "
                             "frame must stay below 2^30 - %d",
                             ldpc::kLanePad);
    }
    // per core column: its state blocks in increasing row order
    std::vector<int32_t> core_first(NC), core_deg(NC, 0), core_state(NS), core_shift(NS);
    for (int i = 0; i < NS; ++i) core_deg[st_core[i]]++;
    for (int k = 0, acc = 0; k < NC; ++k) {
        core_first[k] = acc;
        acc += core_deg[k];
    }
    {
        std::vector<int32_t> fill(NC, 0);
        for (int i = 0; i < NS; ++i) {  // i runs in row-major order, so rows increase
            const int k = st_core[i];
            core_state[core_first[k] + fill[k]] = i;
            core_shift[core_first[k] + fill[k]] = st_shift[i];
            fill[k]++;
        }
    }

    // one device allocation for every table
    const int B = (int)blk_shift.size();
    std::vector<int32_t> host;
    auto put = [&](const std::vector<int32_t> &v) {
        const size_t off = host.size();
        host.insert(host.end(), v.begin(), v.end());
        host.push_back(0);  // keeps every table non-empty
        return off;
    };
    const size_t o_row_first = put(row_first), o_row_deg = put(row_deg), o_row_ns = put(row_ns);
    const size_t o_bs = put(blk_shift), o_bk = put(blk_kind), o_br = put(blk_ref),
                 o_bc = put(blk_col), o_bco = put(blk_core);
    const size_t o_cc = put(core_col), o_cf = put(core_first), o_cd = put(core_deg),
                 o_cs = put(core_state), o_csh = put(core_shift);
    const size_t o_colk = put(col_kind), o_colr = put(col_ref), o_d1s = put(d1_shift),
                 o_d1c = put(d1_col);
    // common rows first: degree <= kSmallRowDegree with at most one degree-1 block
    auto common = [&](int r) {
        return row_deg[r] <= ldpc::kSmallRowDegree && row_ns[r] >= row_deg[r] - 1;
    };
    // common rows grouped by (degree, stored blocks) class, then the others
    auto cls_of = [&](int r) { return 2 * (row_deg[r] - 1) + (row_ns[r] - (row_deg[r] - 1)); };
    std::vector<int32_t> row_list;
    int32_t cls_end[ldpc::kFixedClasses];
    for (int cl = 0; cl < ldpc::kFixedClasses; ++cl) {
        for (int r = 0; r < mb; ++r)
            if (common(r) && cls_of(r) == cl) row_list.push_back(r);
        cls_end[cl] = (int32_t)row_list.size();
    }
    const int n_small = (int)row_list.size();
    for (int r = 0; r < mb; ++r)
        if (!common(r)) row_list.push_back(r);
    const size_t o_rl = put(row_list);
    // degree-1 columns whose row is a common row of degree 3 with 2 stored
    // blocks: that class is updated in the t-domain and takes e^{-|Q|}
    std::vector<int32_t> d1_tdom(d1_col.size(), 0);
    for (size_t k = 0; k < d1_col.size(); ++k)
        d1_tdom[k] = (common(d1_row[k]) && cls_of(d1_row[k]) == ldpc::kTdomClass) ? 1 : 0;
    const size_t o_d1t = put(d1_tdom);
    // descriptors of the common rows (offsets within one frame's arrays)
    const int32_t Zt = ((2 * Z + ldpc::kLanePad) + 63) / 64 * 64;
    const int32_t W = (Z + 63) / 64;
    const int32_t Zp = (Z + 63) / 64 * 64;
    std::vector<int32_t> row_desc((size_t)std::max(n_small, 1) * ldpc::kRowDescWords, 0);
    for (int y = 0; y < n_small; ++y) {
        const int r = row_list[y];
        int32_t *dd = &row_desc[(size_t)y * ldpc::kRowDescWords];
        for (int k = 0; k < row_deg[r]; ++k) {
            const int b = row_first[r] + k;
            if (k < row_ns[r]) {
                dd[k] = blk_core[b] * Zt + blk_shift[b];
                dd[6 + k] = blk_ref[b] * Zp;
            } else {
                dd[12] = blk_ref[b] * Zp;
                dd[13] = blk_ref[b] * W;
                dd[14] = blk_col[b] * Z;
                dd[15] = blk_shift[b];
            }
        }
        dd[16] = r * W;
        dd[17] = r;
        dd[18] = cls_of(r);
    }
    const size_t o_rd = put(row_desc);
    // owner groups: per core column, its owned rows in increasing row order,
    // kGroupRows at a time
    std::vector<int32_t> grp_hdr, grp_desc;
    std::vector<int32_t> core_own(NC, 0), core_ngrp(NC, 0), core_grp0(NC, 0);
    // per core column: its blocks in summation order (owned blocks group by
    // group, then the others), as indices into core_state / core_shift
    std::vector<std::vector<int32_t>> core_order(NC);
    int n_groups = 0;
    for (int k = 0; k < NC; ++k) {
        std::vector<int32_t> own_rows;
        for (int r = 0; r < mb; ++r)
            if (row_owner[r] == core_col[k]) own_rows.push_back(r);
        core_own[k] = (int32_t)own_rows.size();
        core_grp0[k] = n_groups;
        for (size_t i0 = 0; i0 < own_rows.size(); i0 += ldpc::kGroupRows) {
            const int cnt = (int)std::min<size_t>(ldpc::kGroupRows, own_rows.size() - i0);
            grp_hdr.insert(grp_hdr.end(), {k * Zt, cnt, 0, 0});
            for (int i = 0; i < ldpc::kGroupRows; ++i) {
                int32_t dd[ldpc::kGroupDescWords] = {0, 0, 0, 0, 0, 0, 0, 0};
                if (i < cnt) {
                    const int r = own_rows[i0 + i];
                    const int b0 = row_first[r], b1 = b0 + 1, b2 = b0 + 2;
                    dd[0] = blk_ref[b0] * Zp;
                    dd[1] = blk_ref[b1] * Zp;
                    dd[2] = blk_core[b1] * Zt + blk_shift[b1];
                    dd[3] = blk_ref[b2] * Zp;
                    dd[4] = blk_ref[b2] * W;
                    dd[5] = r * W;
                    dd[6] = blk_col[b2] * Z;
                    dd[7] = blk_shift[b2];
                }
                grp_desc.insert(grp_desc.end(), dd, dd + ldpc::kGroupDescWords);
            }
            ++n_groups;
        }
        core_ngrp[k] = n_groups - core_grp0[k];
        // summation order: owned blocks (own_rows order), then the others
        std::vector<int32_t> &ord = core_order[k];
        for (int r : own_rows)
            for (int i = 0; i < core_deg[k]; ++i)
                if (st_row[core_state[core_first[k] + i]] == r) ord.push_back(core_first[k] + i);
        for (int i = 0; i < core_deg[k]; ++i)
            if (row_owner[st_row[core_state[core_first[k] + i]]] != core_col[k])
                ord.push_back(core_first[k] + i);
    }
    int max_half_terms = 1;
    for (int k = 0; k < NC; ++k) {
        const int terms = core_ngrp[k] + core_deg[k] - core_own[k];
        max_half_terms = std::max(max_half_terms, (terms + 1) / 2);
    }
    const size_t o_gh = put(grp_hdr), o_gd = put(grp_desc), o_rot = put(row_rot);
    const size_t o_cown = put(core_own), o_cng = put(core_ngrp), o_cg0 = put(core_grp0);
    // per core column: (message offset, shift) of its blocks at a fixed
    // stride, in summation order
    int max_cd = 1;
    for (int k = 0; k < NC; ++k) max_cd = std::max(max_cd, core_deg[k]);
    const int tab_stride = 2 * max_cd;
    std::vector<int32_t> core_tab((size_t)std::max(NC, 1) * tab_stride, 0);
    for (int k = 0; k < NC; ++k)
        for (int i = 0; i < core_deg[k]; ++i) {
            core_tab[(size_t)k * tab_stride + 2 * i] = core_state[core_order[k][i]] * Zp;
            core_tab[(size_t)k * tab_stride + 2 * i + 1] = core_shift[core_order[k][i]];
        }
    const size_t o_ct = put(core_tab);
    // the same tables in the frame-resident schedule's LDS layout (stride Z)
    std::vector<int32_t> res_desc((size_t)mb * ldpc::kResDescWords, 0);
    for (int r = 0; r < mb; ++r) {
        int32_t *dd = &res_desc[(size_t)r * ldpc::kResDescWords];
        dd[0] = common(r) ? cls_of(r) : (row_deg[r] <= 8 ? 12 : 13);
        dd[1] = row_deg[r];
        dd[2] = row_ns[r];
        dd[3] = row_first[r];
        dd[4] = r * W;
        if (!common(r)) continue;
        for (int k = 0; k < row_deg[r]; ++k) {
            const int b = row_first[r] + k;
            const bool st = k < row_ns[r];
            dd[5 + k] = st ? blk_core[b] * Z : blk_ref[b] * Zp;
            dd[11 + k] = st ? blk_ref[b] * Z : blk_ref[b] * W;
            dd[17 + k] = blk_shift[b];
        }
    }
    const size_t o_resd = put(res_desc);
    // rows padded to whole batches of kResVnBatch pairs, plus one batch of
    // slack, so a batch read from any in-range start stays inside the table
    const int res_batch = 2 * ldpc::kResVnBatch;
    const int res_stride = (tab_stride + res_batch - 1) / res_batch * res_batch;
    std::vector<int32_t> res_core((size_t)std::max(NC, 1) * res_stride + res_batch, 0);
    for (int k = 0; k < NC; ++k)
        for (int i = 0; i < core_deg[k]; ++i) {
            res_core[(size_t)k * res_stride + 2 * i] = core_state[core_order[k][i]] * Z;
            res_core[(size_t)k * res_stride + 2 * i + 1] = core_shift[core_order[k][i]];
        }
    const size_t o_resc = put(res_core);
    // check-phase units in class order (only where a frame could fit in LDS:
    // at most 2^16 units)
    std::vector<int32_t> res_unit;
    if ((int64_t)mb * W <= (1 << 16)) {
        for (int y = 0; y < mb; ++y)
            for (int ch = 0; ch < W; ++ch) res_unit.push_back(row_list[y] | (ch << 16));
    }
    const int32_t n_res_units = (int32_t)res_unit.size();
    const size_t o_resu = put(res_unit);

    ldpc_code *code = new (std::nothrow) ldpc_code();
    if (!code) return fail_with(LDPC_ENOMEM, "host allocation failed");
    hipError_t e = hipGetDevice(&code->device);
    if (e != hipSuccess) {
        delete code;
        return fail_with(LDPC_EDEVICE, "hipGetDevice: %s", hipGetErrorString(e));
    }
    int lds = 0;
    e = hipDeviceGetAttribute(&lds, hipDeviceAttributeMaxSharedMemoryPerBlock, code->device);
    if (e != hipSuccess) {
        delete code;
        return fail_with(LDPC_EDEVICE, "hipDeviceGetAttribute: %s", hipGetErrorString(e));
    }
    code->lds_limit = lds > 0 ? (size_t)lds : 0;
    // the second stream (default priority) and its events; without them every
    // decode runs on the caller's stream alone
    if (hipStreamCreateWithFlags(&code->aux, hipStreamNonBlocking) != hipSuccess ||
        hipEventCreateWithFlags(&code->fork, hipEventDisableTiming) != hipSuccess ||
        hipEventCreateWithFlags(&code->join, hipEventDisableTiming) != hipSuccess) {
        if (code->fork) (void)hipEventDestroy(code->fork);
        if (code->aux) (void)hipStreamDestroy(code->aux);
        code->aux = nullptr;
        code->fork = code->join = nullptr;
    }
    // the capture stream of the decode graphs (default priority); without it
    // every decode launches its kernels one by one
    if (hipStreamCreateWithFlags(&code->cap, hipStreamNonBlocking) != hipSuccess)
        code->cap = nullptr;
    // set-up of the no-allocation decode on this device (its failure is
    // reported by ldpc_decode_batch_noalloc, which retries the lookup)
    (void)scratch_setup(code->device);
    e = hipMalloc(reinterpret_cast<void **>(&code->table), host.size() * sizeof(int32_t));
    if (e != hipSuccess) {
        delete code;
        return fail_with(e == hipErrorOutOfMemory ? LDPC_ENOMEM : LDPC_EDEVICE, "hipMalloc: %s",
                         hipGetErrorString(e));
    }
    e = hipMemcpy(code->table, host.data(), host.size() * sizeof(int32_t), hipMemcpyHostToDevice);
    if (e != hipSuccess) {
        (void)hipFree(code->table);
        delete code;
        return fail_with(LDPC_EDEVICE, "hipMemcpy: %s", hipGetErrorString(e));
    }
    const int32_t *T = code->table;
    CodeDev &d = code->dev;
    d.Z = Z;
    d.mb = mb;
    d.nb = nb;
    d.n = nb * Z;
    d.m = mb * Z;
    d.NS = NS;
    d.NC = NC;
    d.ND1 = ND1;
    d.W = (Z + 63) / 64;
    d.Zt = Zt;
    d.Zp = Zp;
    d.row_first = T + o_row_first;
    d.row_deg = T + o_row_deg;
    d.row_ns = T + o_row_ns;
    d.row_list = T + o_rl;
    d.max_core_deg = 0;
    for (int k = 0; k < NC; ++k) d.max_core_deg = std::max(d.max_core_deg, core_deg[k]);
    d.n_small = n_small;
    d.n_large = mb - n_small;
    for (int cl = 0; cl < ldpc::kFixedClasses; ++cl) d.cls_end[cl] = cls_end[cl];
    d.row_desc = T + o_rd;
    d.blk_shift = T + o_bs;
    d.blk_kind = T + o_bk;
    d.blk_ref = T + o_br;
    d.blk_col = T + o_bc;
    d.blk_core = T + o_bco;
    d.core_col = T + o_cc;
    d.core_first = T + o_cf;
    d.core_deg = T + o_cd;
    d.core_state = T + o_cs;
    d.core_shift = T + o_csh;
    d.core_tab = T + o_ct;
    d.core_tab_stride = tab_stride;
    d.res_desc = T + o_resd;
    d.res_core = T + o_resc;
    d.res_core_stride = res_stride;
    d.res_unit = T + o_resu;
    d.res_units = n_res_units;
    d.col_kind = T + o_colk;
    d.col_ref = T + o_colr;
    d.d1_shift = T + o_d1s;
    d.d1_col = T + o_d1c;
    d.d1_tdom = T + o_d1t;
    d.row_rot = T + o_rot;
    d.n_groups = n_groups;
    d.n_tdom = cls_end[ldpc::kTdomClass] - cls_end[ldpc::kTdomClass - 1];
    d.grp_hdr = T + o_gh;
    d.grp_desc = T + o_gd;
    d.core_own = T + o_cown;
    d.core_ngrp = T + o_cng;
    d.core_grp0 = T + o_cg0;
    d.max_half_terms = max_half_terms;

    ldpc_code_info_t &I = code->info;
    I.n = d.n;
    I.m = d.m;
    I.Z = Z;
    I.mb = mb;
    I.nb = nb;
    I.blocks = B;
    I.edges = (int64_t)B * Z;
    I.state_edges = (int64_t)NS * Z;
    I.core_cols = NC;
    I.deg1_cols = ND1;
    I.deg0_cols = nb - NC - ND1;
    I.max_row_degree = maxdeg;
    int64_t owned = 0;
    for (int k = 0; k < NC; ++k) owned += core_own[k];
    I.owned_edges = owned * Z;
    I.owner_groups = n_groups;
    *out = code;
    return LDPC_OK;
}

void ldpc_code_destroy(ldpc_code *code) {
    if (!code) return;
    for (auto &g : code->graphs)
        if (g.exec) (void)hipGraphExecDestroy(g.exec);
    if (code->cap) (void)hipStreamDestroy(code->cap);
    if (code->aux) (void)hipStreamSynchronize(code->aux);
    if (code->join) (void)hipEventDestroy(code->join);
    if (code->fork) (void)hipEventDestroy(code->fork);
    if (code->aux) (void)hipStreamDestroy(code->aux);
    if (code->table) (void)hipFree(code->table);
    delete code;
}

int ldpc_code_info(const ldpc_code *code, ldpc_code_info_t *out) {
    if (!code || !out) return fail_with(LDPC_EINVAL, "null argument");
    *out = code->info;
    return LDPC_OK;
}

size_t ldpc_workspace_bytes(const ldpc_code *code, int32_t F, int32_t max_iters,
                            const ldpc_decode_opts *opts) {
    if (!code || F < 1 || max_iters < 0) return 0;
    ldpc_decode_opts o;
    ldpc_decode_opts_init(&o);
    if (opts) o = *opts;
    return ldpc::decode_workspace_bytes(code->dev, F, max_iters, o.msg_fp16 != 0,
                                        o.llr_out != nullptr);
}

}  // extern "C"

namespace {

// The schedule a decode of F frames with options o runs on: the resident one
// needs no posterior output and no per-pass events, and the frame's state
// must fit in one workgroup's LDS.  Automatic choice by a cost model per
// iteration, fitted to measurements on MI355X: the resident schedule takes
// about kResidentUnitNs per (base row, 64 checks) unit of a frame, for every
// round of up to kResidentFramesPerRound frames (one workgroup per CU); the
// launches (one stream) take kLaunchFixedNs plus kLaunchWgNs per workgroup of
// the two passes: check items of one owner group over 256 positions or of one
// other row over 256 * cpt checks, variable items of 512 variables.  On the
// rate-0.02 template at Z = 64 (15 check and 6 variable items per frame) the
// launches measured 10.1, 13.8, 27.3 and 75 us per iteration at 16, 64, 256
// and 1024 frames, the resident schedule 11.4-11.6 us per round.
constexpr double kResidentUnitNs = 80.0;
constexpr int kResidentFramesPerRound = 256;
constexpr double kLaunchFixedNs = 8800.0;
constexpr double kLaunchWgNs = 3.2;

bool resident_pays(const CodeDev &c, int F, int cpt) {
    const double units = (double)c.mb * c.W;
    const double rounds = (double)((F + kResidentFramesPerRound - 1) / kResidentFramesPerRound);
    const double t_res = rounds * units * kResidentUnitNs;
    const int gt = (c.Z + 255) / 256, rt = (c.Z + 256 * cpt - 1) / (256 * cpt);
    const int grouped_rows = c.n_groups > 0 ? c.n_tdom : 0;
    const double check = (double)c.n_groups * gt + (double)(c.mb - grouped_rows) * rt;
    const double var = (double)c.NC * ((c.Z + 511) / 512);
    return t_res < kLaunchFixedNs + kLaunchWgNs * (double)F * (check + var);
}

// Checks per thread when the caller leaves the choice to the library: 1 for
// liftings of at most 256 (a row's checks fit one 256-thread tile anyway, and
// lighter workgroups measured 7-11% faster there), else 4.
int default_cpt(const CodeDev &c) { return c.Z <= 256 ? 1 : ldpc::kDefaultChecksPerThread; }

int resolve_schedule(const ldpc_code *code, int F, const ldpc_decode_opts &o, int *out) {
    if (o.checks_per_thread != 0 && o.checks_per_thread != 1 && o.checks_per_thread != 2 &&
        o.checks_per_thread != 4)
        return fail_with(LDPC_EINVAL, "checks_per_thread = %d is not 0, 1, 2 or 4",
                         o.checks_per_thread);
    if (o.schedule < LDPC_SCHEDULE_AUTO || o.schedule > LDPC_SCHEDULE_SPLIT)
        return fail_with(LDPC_EINVAL, "schedule = %d is not 0, 1, 2 or 3", o.schedule);
    if (o.schedule == LDPC_SCHEDULE_SPLIT &&
        (o.llr_out || o.timing_events || F > ldpc::kSplitMaxFrames ||
         !ldpc::split_offered(code->dev, o.msg_fp16 != 0)))
        return fail_with(LDPC_EUNSUPPORTED,
                         "split schedule: needs llr_out and timing_events unset, at most %d "
                         "frames and a frame state of at most %zu bytes",
                         ldpc::kSplitMaxFrames, ldpc::kSplitMaxStateBytes);
    const bool possible = !o.llr_out && !o.timing_events && code->dev.res_units > 0 &&
                          ldpc::resident_layout(code->dev, o.msg_fp16 != 0).total <= code->lds_limit;
    if (o.schedule == LDPC_SCHEDULE_RESIDENT && !possible)
        return fail_with(LDPC_EUNSUPPORTED,
                         "resident schedule: needs llr_out and timing_events unset and %zu LDS "
                         "bytes (limit %zu)",
                         ldpc::resident_layout(code->dev, o.msg_fp16 != 0).total, code->lds_limit);
    if (o.schedule == LDPC_SCHEDULE_AUTO)
        *out = (possible && resident_pays(code->dev, F, o.checks_per_thread == 0
                                                            ? default_cpt(code->dev)
                                                            : o.checks_per_thread))
                   ? LDPC_SCHEDULE_RESIDENT
                   : LDPC_SCHEDULE_LAUNCHES;
    else
        *out = o.schedule;
    return LDPC_OK;
}

}  // namespace

extern "C" {

int ldpc_decode_schedule(const ldpc_code *code, int32_t F, const ldpc_decode_opts *opts,
                         int32_t *schedule_out) {
    if (!code || !schedule_out) return fail_with(LDPC_EINVAL, "null pointer");
    if (F < 1 || F > 65535) return fail_with(LDPC_EINVAL, "F = %d outside [1, 65535]", F);
    ldpc_decode_opts o;
    ldpc_decode_opts_init(&o);
    if (opts) o = *opts;
    int sched = 0;
    const int st = resolve_schedule(code, F, o, &sched);
    if (st != LDPC_OK) return st;
    *schedule_out = sched;
    return LDPC_OK;
}

}  // extern "C"

namespace {

// Edge visits per iteration, F x (stored + degree-1 blocks) x Z, from which the
// per-iteration launches run the frames as two halves on two streams by
// default.  Two streams double the launches of an iteration, so a decode whose
// iterations are short runs into the launch rate: 100 iterations take at least
// about 1.05 ms on two streams against 0.63 ms on one.  Measured on the
// rate-0.02 and rate-0.05 templates at Z = 2048 to 6667 and 2 to 16 frames,
// 100 iterations, one decode repeated: two streams faster from 14.7M visits
// with float32 messages and from 12M with half, one stream faster or level
// below (by up to 40% at 2M-6M).  A stream of different decodes submitted back
// to back gains less: the host's launches overlap the previous decode's GPU
// work only while the GPU is the bottleneck, and once frames converge it is
// not.  Nine rate-0.02/0.05/0.1 decodes of 7-8 frames in sequence ran at 2094
// Mbit/s with thresholds of 14M / 12M and at 2354 with 24M / 16M, and the
// 8-frame n = 1,000,050 decode (24.0M) gained 8-11% from two streams.
constexpr int64_t kTwoStreamEdgesF32 = 24000000;
constexpr int64_t kTwoStreamEdgesF16 = 16000000;

bool two_streams(const ldpc_code *code, int F, const ldpc_decode_opts &o) {
    if (F < 2 || o.timing_events || o.streams == 1) return false;
    if (o.streams == 2) return true;
    const int64_t edges = (int64_t)F * (code->dev.NS + code->dev.ND1) * code->dev.Z;
    return edges >= (o.msg_fp16 ? kTwoStreamEdgesF16 : kTwoStreamEdgesF32);
}

// The words that identify a decode for the graph cache: everything a
// captured launch sequence bakes in (sizes, options, pointers, stream mode).
void graph_key(const ldpc::DecodeLaunch &l, bool two, int64_t (&k)[ldpc_code::kGraphKeyWords]) {
    int i = 0;
    k[i++] = l.F;
    k[i++] = l.T;
    k[i++] = l.early_stop;
    k[i++] = l.check_from;
    k[i++] = l.fp16;
    k[i++] = l.cpt;
    k[i++] = two ? 1 : 0;
    k[i++] = (int64_t)(uintptr_t)l.llr;
    k[i++] = (int64_t)(uintptr_t)l.syndrome;
    k[i++] = (int64_t)(uintptr_t)l.bits_out;
    k[i++] = (int64_t)(uintptr_t)l.iters_out;
    k[i++] = (int64_t)(uintptr_t)l.conv_out;
    k[i++] = (int64_t)(uintptr_t)l.llr_out;
    k[i++] = (int64_t)(uintptr_t)l.ws;
    while (i < ldpc_code::kGraphKeyWords) k[i++] = 0;
}

// Enqueue a decode on the per-iteration launches through the code's graph
// cache (caller holds aux_lock): replay the cached graph of this exact call,
// capture it at the key's second call, else launch the kernels directly.  A
// failed capture falls back to direct launches for that key.
hipError_t graph_decode(ldpc_code *mc, ldpc::DecodeLaunch l, bool two) {
    int64_t key[ldpc_code::kGraphKeyWords];
    graph_key(l, two, key);
    ldpc_code::GraphSlot *s = nullptr;
    for (auto &g : mc->graphs)
        if (std::equal(key, key + ldpc_code::kGraphKeyWords, g.key)) s = &g;
    if (!s) {
        s = &mc->graphs[0];
        for (auto &g : mc->graphs)
            if (g.used < s->used) s = &g;
        if (s->exec) (void)hipGraphExecDestroy(s->exec);
        *s = ldpc_code::GraphSlot{};
        std::copy(key, key + ldpc_code::kGraphKeyWords, s->key);
    }
    s->used = ++mc->graph_clock;
    if (!s->exec) {
        if (s->seen < 0 || ++s->seen < 2 || !mc->cap) return ldpc::enqueue_decode(l);
        const hipStream_t caller = l.stream;
        l.stream = mc->cap;
        hipGraph_t graph = nullptr;
        hipError_t e = hipStreamBeginCapture(mc->cap, hipStreamCaptureModeThreadLocal);
        if (e == hipSuccess) {
            const hipError_t el = ldpc::enqueue_decode(l);
            e = hipStreamEndCapture(mc->cap, &graph);
            if (el != hipSuccess) e = el;
        }
        if (e == hipSuccess) e = hipGraphInstantiate(&s->exec, graph, nullptr, nullptr, 0);
        if (graph) (void)hipGraphDestroy(graph);
        l.stream = caller;
        if (e != hipSuccess) {
            (void)hipGetLastError();
            s->exec = nullptr;
            s->seen = -1;
            return ldpc::enqueue_decode(l);
        }
    }
    return hipGraphLaunch(s->exec, l.stream);
}

// Edge visits per iteration up to which a repeated decode is replayed from a
// graph.  Graphs pay where the host's two launches per iteration take about
// as long as the iteration itself: 16 frames of the n = 9,600 rate-0.02 code
// (0.46M visits) went from 1.01 to 0.90 ms per decode.  A larger decode is
// bound by the GPU, and replaying it gains nothing and costs a little: nine
// different decodes of 1.3M-24M visits in sequence ran 3% slower (2194-2260
// against 2317-2326 Mbit/s), and two-stream decodes lost their overlap in
// part (8 frames of n = 1,000,050 with FP16 messages -1.7%, 32 frames -3%).
constexpr int64_t kGraphMaxEdges = 1000000;

bool graph_pays(const ldpc_code *code, int F, bool two) {
    const int64_t edges = (int64_t)F * (code->dev.NS + code->dev.ND1) * code->dev.Z;
    return !two && edges <= kGraphMaxEdges;
}

// Whether `stream` is being captured by its owner (then the kernels go into
// that capture one by one).  A failed query counts as capturing.
bool stream_capturing(hipStream_t stream) {
    hipStreamCaptureStatus st = hipStreamCaptureStatusNone;
    if (hipStreamIsCapturing(stream, &st) != hipSuccess) return true;
    return st != hipStreamCaptureStatusNone;
}

// The body of both decode entry points.  noalloc: `workspace` is ignored and
// the decode runs in the device's fixed scratch region.
int decode_batch_impl(const ldpc_code *code, int32_t F, const float *llr, const uint8_t *syndrome,
                      int32_t max_iters, uint8_t *bits_out, int32_t *iters_out,
                      uint8_t *converged_out, const ldpc_decode_opts *opts, void *workspace,
                      size_t workspace_bytes, void *stream, bool noalloc) {
    if (!code) return fail_with(LDPC_EINVAL, "code is null");
    if (F < 1 || F > 65535) return fail_with(LDPC_EINVAL, "F = %d outside [1, 65535]", F);
    if (max_iters < 0) return fail_with(LDPC_EINVAL, "max_iters = %d < 0", max_iters);
    if (!llr || !syndrome || !bits_out || !iters_out || !converged_out)
        return fail_with(LDPC_EINVAL, "null input or output pointer");
    ldpc_decode_opts o;
    ldpc_decode_opts_init(&o);
    if (opts) o = *opts;
    const int cpt = o.checks_per_thread == 0 ? default_cpt(code->dev) : o.checks_per_thread;
    if (cpt != 1 && cpt != 2 && cpt != 4)
        return fail_with(LDPC_EINVAL, "checks_per_thread = %d is not 0, 1, 2 or 4",
                         o.checks_per_thread);
    if (o.check_from_iter < 0) return fail_with(LDPC_EINVAL, "check_from_iter < 0");
    if (o.streams < 0 || o.streams > 2)
        return fail_with(LDPC_EINVAL, "streams = %d is not 0, 1 or 2", o.streams);
    if (o.graphs < 0 || o.graphs > 1)
        return fail_with(LDPC_EINVAL, "graphs = %d is not 0 or 1", o.graphs);
    if (o.timing_events && (int64_t)o.n_timing_events < 4ll * max_iters)
        return fail_with(LDPC_EINVAL, "%d timing events; need 4*max_iters = %lld",
                         o.n_timing_events, 4ll * max_iters);
    if ((int64_t)(max_iters + 1) * F >= (1ll << 31))
        return fail_with(LDPC_EINVAL, "(max_iters + 1) * F too large");
    const size_t need = ldpc::decode_workspace_bytes(code->dev, F, max_iters, o.msg_fp16 != 0,
                                                     o.llr_out != nullptr);
    if (noalloc) {
        if (need > kScratchBytes)
            return fail_with(LDPC_EWORKSPACE,
                             "decode needs %zu bytes of state; the no-allocation scratch region "
                             "holds %zu (fewer frames or iterations per call)",
                             need, kScratchBytes);
    } else if (!workspace || workspace_bytes < need ||
               (reinterpret_cast<uintptr_t>(workspace) & 255)) {
        return fail_with(LDPC_EWORKSPACE, "workspace %p of %zu bytes; need %zu bytes, 256-aligned",
                         workspace, workspace_bytes, need);
    }
    int sched = 0;
    int st = resolve_schedule(code, F, o, &sched);
    if (st != LDPC_OK) return st;
    st = check_device(code);
    if (st != LDPC_OK) return st;
    if (noalloc) {
        workspace = scratch_ptr(code->device);
        if (!workspace) {
            const hipError_t e = scratch_setup(code->device);
            if (e != hipSuccess)
                return fail_with(LDPC_EDEVICE, "scratch region: hipGetSymbolAddress: %s",
                                 hipGetErrorString(e));
            workspace = scratch_ptr(code->device);
        }
    }

    ldpc::DecodeLaunch l{};
    l.c = code->dev;
    l.F = F;
    l.T = max_iters;
    l.early_stop = o.early_stop ? 1 : 0;
    l.check_from = o.check_from_iter;
    l.fp16 = o.msg_fp16 ? 1 : 0;
    l.cpt = cpt;
    l.llr = llr;
    l.syndrome = syndrome;
    l.bits_out = bits_out;
    l.iters_out = iters_out;
    l.conv_out = converged_out;
    l.llr_out = o.llr_out;
    l.ws = static_cast<char *>(workspace);
    l.events = reinterpret_cast<hipEvent_t *>(o.timing_events);
    l.stream = static_cast<hipStream_t>(stream);
    const ldpc::WorkLayout WL = ldpc::work_layout(l.c, F, max_iters, l.fp16 != 0, false);
    hipError_t e;
    if (sched == LDPC_SCHEDULE_RESIDENT) {
        e = ldpc::enqueue_resident(l, WL, code->lds_limit);
    } else if (sched == LDPC_SCHEDULE_SPLIT) {
        e = ldpc::enqueue_split(l, WL);
    } else {
        ldpc_code *mc = const_cast<ldpc_code *>(code);
        const bool two = two_streams(code, F, o);
        const bool graph = !noalloc && o.graphs == 0 && !l.events && graph_pays(code, F, two) &&
                           !stream_capturing(l.stream);
        std::lock_guard<std::mutex> g(mc->aux_lock);
        if (two) {
            l.aux = mc->aux;
            l.fork = mc->fork;
            l.join = mc->join;
        }
        e = graph ? graph_decode(mc, l, two) : ldpc::enqueue_decode(l);
    }
    if (e != hipSuccess) return fail_with(LDPC_EDEVICE, "launch: %s", hipGetErrorString(e));
    return LDPC_OK;
}

}  // namespace

extern "C" {

int ldpc_decode_batch(const ldpc_code *code, int32_t F, const float *llr, const uint8_t *syndrome,
                      int32_t max_iters, uint8_t *bits_out, int32_t *iters_out,
                      uint8_t *converged_out, const ldpc_decode_opts *opts, void *workspace,
                      size_t workspace_bytes, void *stream) {
    return decode_batch_impl(code, F, llr, syndrome, max_iters, bits_out, iters_out, converged_out,
                             opts, workspace, workspace_bytes, stream, false);
}

int ldpc_decode_batch_noalloc(const ldpc_code *code, int32_t F, const float *llr,
                              const uint8_t *syndrome, int32_t max_iters, uint8_t *bits_out,
                              int32_t *iters_out, uint8_t *converged_out,
                              const ldpc_decode_opts *opts, void *stream) {
    return decode_batch_impl(code, F, llr, syndrome, max_iters, bits_out, iters_out, converged_out,
                             opts, nullptr, 0, stream, true);
}

int ldpc_syndrome(const ldpc_code *code, int32_t F, const uint8_t *bits, uint8_t *syn_out,
                  void *stream) {
    if (!code) return fail_with(LDPC_EINVAL, "code is null");
    if (F < 1 || F > 65535) return fail_with(LDPC_EINVAL, "F = %d outside [1, 65535]", F);
    if (!bits || !syn_out) return fail_with(LDPC_EINVAL, "null pointer");
    int st = check_device(code);
    if (st != LDPC_OK) return st;
    hipError_t e = ldpc::enqueue_syndrome(code->dev, F, bits, syn_out,
                                          static_cast<hipStream_t>(stream));
    if (e != hipSuccess) return fail_with(LDPC_EDEVICE, "launch: %s", hipGetErrorString(e));
    return LDPC_OK;
}

static bool valid_dim(int d) { return d == 1 || d == 2 || d == 4 || d == 8; }

int ldpc_reconciliation_llr(int32_t d, int32_t F, int32_t n, const float *x, const float *m,
                            float sigma2, float *llr_out, void *stream) {
    if (!valid_dim(d)) return fail_with(LDPC_EINVAL, "d = %d is not 1, 2, 4 or 8", d);
    if (F < 1 || F > 65535 || n < 1) return fail_with(LDPC_EINVAL, "F = %d, n = %d", F, n);
    if ((int64_t)n + d >= (1ll << 31)) return fail_with(LDPC_EINVAL, "n too large");
    if (!(sigma2 > 0.0f)) return fail_with(LDPC_EINVAL, "sigma2 must be > 0");
    if (!x || !m || !llr_out) return fail_with(LDPC_EINVAL, "null pointer");
    hipError_t e = ldpc::enqueue_reconciliation_llr(d, F, n, x, m, sigma2, llr_out,
                                                    static_cast<hipStream_t>(stream));
    if (e != hipSuccess) return fail_with(LDPC_EDEVICE, "launch: %s", hipGetErrorString(e));
    return LDPC_OK;
}

int ldpc_reconciliation_message(int32_t d, int32_t F, int32_t n, const uint8_t *bits,
                                const float *y, float *m_out, void *stream) {
    if (!valid_dim(d)) return fail_with(LDPC_EINVAL, "d = %d is not 1, 2, 4 or 8", d);
    if (F < 1 || F > 65535 || n < 1) return fail_with(LDPC_EINVAL, "F = %d, n = %d", F, n);
    if ((int64_t)n + d >= (1ll << 31)) return fail_with(LDPC_EINVAL, "n too large");
    if (!bits || !y || !m_out) return fail_with(LDPC_EINVAL, "null pointer");
    hipError_t e = ldpc::enqueue_reconciliation_message(d, F, n, bits, y, m_out,
                                                        static_cast<hipStream_t>(stream));
    if (e != hipSuccess) return fail_with(LDPC_EDEVICE, "launch: %s", hipGetErrorString(e));
    return LDPC_OK;
}

struct ldpc_engine {
    ldpc::Engine e;
};

int ldpc_engine_create(const ldpc_engine_config *cfg, ldpc_engine **out) {
    if (!out) return fail_with(LDPC_EINVAL, "out is null");
    *out = nullptr;
    if (!cfg) return fail_with(LDPC_EINVAL, "cfg is null");
    if (cfg->hbm_budget_bytes == 0) return fail_with(LDPC_EINVAL, "hbm_budget_bytes is 0");
    if (cfg->max_slots < 1 || cfg->max_slots > ldpc::kEngineMaxSlots)
        return fail_with(LDPC_EINVAL, "max_slots = %d outside 1..%d", cfg->max_slots,
                         ldpc::kEngineMaxSlots);
    const int cpt = cfg->checks_per_thread == 0 ? ldpc::kDefaultChecksPerThread : cfg->checks_per_thread;
    if (cpt != 1 && cpt != 2 && cpt != 4)
        return fail_with(LDPC_EINVAL, "checks_per_thread = %d is not 0, 1, 2 or 4",
                         cfg->checks_per_thread);
    if (cfg->max_step_edges < 0)
        return fail_with(LDPC_EINVAL, "max_step_edges = %lld is negative",
                         (long long)cfg->max_step_edges);
    ldpc_engine *en = new (std::nothrow) ldpc_engine();
    if (!en) return fail_with(LDPC_ENOMEM, "host allocation failed");
    en->e.max_step_edges = cfg->max_step_edges;
    hipError_t e = hipGetDevice(&en->e.device);
    if (e == hipSuccess)
        e = en->e.init(cfg->hbm_budget_bytes, cfg->max_slots, cfg->msg_fp16 != 0,
                       cfg->early_stop != 0, cpt, cfg->stream);
    if (e != hipSuccess) {
        en->e.destroy();
        delete en;
        return fail_with(e == hipErrorOutOfMemory ? LDPC_ENOMEM : LDPC_EDEVICE, "engine: %s",
                         hipGetErrorString(e));
    }
    *out = en;
    return LDPC_OK;
}

void ldpc_engine_destroy(ldpc_engine *en) {
    if (!en) return;
    en->e.destroy();
    delete en;
}

size_t ldpc_engine_request_bytes(const ldpc_code *code, int32_t F, int32_t max_iters,
                                 int32_t msg_fp16) {
    if (!code || F < 1 || max_iters < 0) return 0;
    return ldpc::Engine::request_bytes(code->dev, F, max_iters, msg_fp16 != 0);
}

int ldpc_engine_submit(ldpc_engine *en, const ldpc_code *code, int32_t F, const float *llr,
                       const uint8_t *syndrome, int32_t max_iters, uint8_t *bits_out,
                       int32_t *iters_out, uint8_t *converged_out, int64_t *ticket_out) {
    if (!en || !code || !ticket_out) return fail_with(LDPC_EINVAL, "null engine, code or ticket");
    if (F < 1 || F > 65535) return fail_with(LDPC_EINVAL, "F = %d outside [1, 65535]", F);
    if (max_iters < 0) return fail_with(LDPC_EINVAL, "max_iters = %d < 0", max_iters);
    if (!llr || !syndrome || !bits_out || !iters_out || !converged_out)
        return fail_with(LDPC_EINVAL, "null input or output pointer");
    if ((int64_t)(max_iters + 1) * F >= (1ll << 31))
        return fail_with(LDPC_EINVAL, "(max_iters + 1) * F too large");
    if (code->dev.n_large > 0)
        return fail_with(LDPC_EUNSUPPORTED,
                         "the engine takes codes whose rows have degree <= %d and at most one "
                         "degree-1 block", ldpc::kSmallRowDegree);
    if (code->device != en->e.device)
        return fail_with(LDPC_EDEVICE, "code on device %d, engine on device %d", code->device,
                         en->e.device);
    const size_t need = ldpc::Engine::request_bytes(code->dev, F, max_iters, en->e.fp16);
    if (need > en->e.budget_bytes)
        return fail_with(LDPC_EINVAL, "request needs %zu bytes, budget is %zu", need,
                         en->e.budget_bytes);
    ldpc::Request r{};
    r.c = code->dev;
    r.F = F;
    r.T = max_iters;
    r.llr = llr;
    r.syndrome = syndrome;
    r.bits_out = bits_out;
    r.iters_out = iters_out;
    r.conv_out = converged_out;
    *ticket_out = en->e.submit(r);
    return LDPC_OK;
}

int ldpc_engine_step(ldpc_engine *en, int32_t *active_out, int32_t *queued_out) {
    if (!en) return fail_with(LDPC_EINVAL, "engine is null");
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev != en->e.device)
        return fail_with(LDPC_EDEVICE, "current device is not the engine's device");
    int a = 0, q = 0;
    hipError_t e = en->e.step(&a, &q);
    if (active_out) *active_out = a;
    if (queued_out) *queued_out = q;
    if (e != hipSuccess) return fail_with(LDPC_EDEVICE, "engine step: %s", hipGetErrorString(e));
    return LDPC_OK;
}

int ldpc_engine_poll(ldpc_engine *en, int64_t *tickets_out, int32_t capacity, int32_t *count_out) {
    if (!en || !count_out || (capacity > 0 && !tickets_out))
        return fail_with(LDPC_EINVAL, "null argument");
    *count_out = capacity > 0 ? en->e.poll(tickets_out, capacity) : 0;
    return LDPC_OK;
}

}  // extern "C"
