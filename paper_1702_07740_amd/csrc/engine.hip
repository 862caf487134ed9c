// Multi-request decode engine: iteration-level scheduling of many requests of
// mixed codes on one stream, gfx950.
//
// A request (F frames of one code, its own max_iters) is admitted into a slot
// when a slot is free and its decode state fits the engine's HBM budget; its
// state lives in a device arena until it retires.  Every engine step runs ONE
// iteration of every active slot with two launches that cover all slots: the
// check pass (each slot in its own mode: first iteration, steady, or the
// vote-only pass after its last iteration) and the variable pass.  So a
// request arriving while others decode joins the running batch at the next
// step, and small requests share the device with large ones instead of
// queueing behind them.
//
// Per frame, the engine runs exactly the kernel sequence ldpc_decode_batch
// runs (the same device code from passes.h, in the same order), so a
// request's outputs are bit-identical to decoding it alone.
//
// Retirement.  After each step a status kernel counts, per slot, the frames
// whose parity check has not yet succeeded, and the counts are copied to pinned
// host memory asynchronously.  The host retires a slot (read-out kernel, then
// its arena space is reused) once its count reaches 0 or it has run its final
// vote; it learns this a few steps late at most, and meanwhile the kernels skip
// the slot's finished frames.
#include "engine.h"
#include "passes.h"

#include <algorithm>
#include <cstring>
#include <deque>
#include <vector>

namespace ldpc {

namespace {

using namespace dev;

constexpr int kStatusRing = 4;

// What a work item needs before its first dependent load, per active slot,
// in the kernel arguments: with these a workgroup issues its row descriptor
// (check pass) or column table (variable pass) and its flag loads together
// with the loads of the slot's full descriptor, instead of after them.
struct SlotHead {
    const int32_t *tab;  // check pass: the code's row descriptors; variable pass: core_tab
    int32_t *fail;
    int32_t tiles;       // work tiles per row (check pass) or per core column (variable pass)
    int32_t rows;        // check pass: rows with their own items; variable pass: NC
    int32_t start_step, T, F, stride;  // stride: core_tab_stride (variable pass)
    // check pass, per frame: rows x tiles row items, then gitems owner-group
    // items (gtiles per group); in the vote-only step gitems = 0 and every
    // row has row items
    int32_t gitems, gtiles;
};

// Work-item offsets by slot and the slot heads, in the kernel arguments.
struct SlotIndex {
    int n;
    int begin[kEngineMaxSlots + 1];
    SlotHead head[kEngineMaxSlots];
};

// The slot of a work item: the largest s with begin[s] <= item.  Lane l tests
// begin[l + 1] (one load per lane, one ballot), so the lookup costs one
// memory round trip instead of a chain of dependent loads.
__device__ __forceinline__ int find_slot(const SlotIndex &ix, int item) {
    const int l = (int)(threadIdx.x & 63);
    const int b = ix.begin[l + 1];
    return __popcll(__ballot(l + 1 < ix.n && b <= item));
}

__device__ __forceinline__ bool checked_iter(const SlotDesc &S, int t) {
    return t == S.T || (S.early_stop && t >= S.check_from);
}

template <typename Msg, int CPT>
__global__ __launch_bounds__(kBlock) void engine_check_pass(const SlotDesc *slots, SlotIndex ix,
                                                            int step) {
    const int item = (int)xcd_item(blockIdx.x, (unsigned)ix.begin[ix.n]);
    if (item >= ix.begin[ix.n]) return;
    const int s = find_slot(ix, item);
    const SlotHead &H = ix.head[s];
    const int t = step - H.start_step + 1;
    if (t < 1 || t > H.T + 1) return;
    const int local = item - ix.begin[s];
    const int per_frame = H.gitems + H.rows * H.tiles;
    const int f = local / per_frame;
    const int r0 = local - f * per_frame;
    // the row items run first (they carry the most work per check), then the
    // owner-group items; r is the position with the group items first
    const int row_items = per_frame - H.gitems;
    const int r = r0 < row_items ? r0 + H.gitems : r0 - row_items;
    const bool vote_only = t == H.T + 1;
    const SlotDesc &S = slots[s];
    CnArgs A{};
    A.llr = S.llr;
    A.psi = S.psi;
    A.msg = S.msg;
    A.tot = S.tot;
    A.synbits = S.synbits;
    A.fail = H.fail;
    A.d1post = nullptr;
    A.msg_frame = S.L.msg_frame;
    A.tot_frame = S.L.tot_frame;
    A.d1_frame = S.L.d1bits_frame;
    A.syn_frame = S.L.synbits_frame;
    A.psi_frame = S.L.psi_frame;
    A.part = S.part;
    A.part_frame = S.L.part_frame;
    A.F = H.F;
    if (vote_only) {
        A.t = H.T;
        A.vote = 1;
        A.d1_from_llr = H.T == 0;
        A.d1_prev = S.d1b[H.T & 1];
        A.d1_cur = nullptr;
        A.skip_after = H.T >= 1 ? H.T - 1 : -1;
    } else {
        A.t = t;
        A.vote = checked_iter(S, t - 1) ? 1 : 0;
        A.d1_from_llr = t == 1;
        A.d1_prev = S.d1b[(t - 1) & 1];
        A.d1_cur = S.d1b[t & 1];
        A.skip_after = t >= 2 ? t - 2 : -1;
    }
    // the row descriptor through the slot head (its address needs no slot load)
    CodeDev c = S.c;
    c.row_desc = H.tab;
    if (r < H.gitems) {
        // an owner group (never in the vote-only step)
        const int g = r / H.gtiles;
        const unsigned tile = (unsigned)(r - g * H.gtiles);
        if (t == 1)
            group_work<kFirst, Msg>(c, A, f, g, tile);
        else
            group_work<kSteady, Msg>(c, A, f, g, tile);
        return;
    }
    const int r2 = r - H.gitems;
    const int y0 = r2 / H.tiles;
    const unsigned tile = (unsigned)(r2 - y0 * H.tiles);
    // row_list position (every row of an engine code is common); outside the
    // vote-only step the t-domain rows belong to the owner groups
    const int lo = c.cls_end[kTdomClass - 1];
    const int y = (vote_only || y0 < lo) ? y0 : y0 + c.n_tdom;
    if (vote_only)
        check_work_by_desc<Msg, kVoteOnly, CPT>(c, A, f, y, tile);
    else if (t == 1)
        check_work_by_desc<Msg, kFirst, CPT>(c, A, f, y, tile);
    else
        check_work_by_desc<Msg, kSteady, CPT>(c, A, f, y, tile);
}

// The variable pass over all slots (two variables per thread, reading the
// owner-group partials the check pass wrote), with the batch width of the
// largest column among them.
template <typename Msg, int U>
__global__ __launch_bounds__(kBlock) void engine_variable_pass(const SlotDesc *slots, SlotIndex ix,
                                                               int step) {
    const int item = (int)xcd_item(blockIdx.x, (unsigned)ix.begin[ix.n]);
    if (item >= ix.begin[ix.n]) return;
    const int s = find_slot(ix, item);
    const SlotHead &H = ix.head[s];
    const int t = step - H.start_step + 1;
    if (t < 1 || t > H.T) return;
    int local = item - ix.begin[s];
    const unsigned tile = (unsigned)(local % H.tiles);
    local /= H.tiles;
    const int k = local % H.rows;
    const int f = local / H.rows;
    if (uniform_i32(H.fail + (size_t)(t - 1) * H.F + f) == 0) return;
    const SlotDesc &S = slots[s];
    VnArgs V{};
    V.llr = S.llr;
    V.msg = S.msg;
    V.tot = S.tot;
    V.fail = H.fail;
    V.msg_frame = S.L.msg_frame;
    V.tot_frame = S.L.tot_frame;
    V.part = S.part;
    V.part_frame = S.L.part_frame;
    V.F = H.F;
    V.t = t;
    // the column table through the slot head (its address needs no slot load)
    CodeDev c = S.c;
    c.core_tab = H.tab;
    c.core_tab_stride = H.stride;
    variable_work<U, Msg, vn_vpt<Msg>(), true>(c, V, f, k, tile);
}

template <typename Msg>
void launch_engine_variable(dim3 g, dim3 b, hipStream_t st, const SlotDesc *slots, SlotIndex ix,
                            int step, int max_deg) {
    switch (variable_group(max_deg)) {
        case 4: engine_variable_pass<Msg, 4><<<g, b, 0, st>>>(slots, ix, step); break;
        case 8: engine_variable_pass<Msg, 8><<<g, b, 0, st>>>(slots, ix, step); break;
        case 13: engine_variable_pass<Msg, 13><<<g, b, 0, st>>>(slots, ix, step); break;
        case 16: engine_variable_pass<Msg, 16><<<g, b, 0, st>>>(slots, ix, step); break;
        default: engine_variable_pass<Msg, 26><<<g, b, 0, st>>>(slots, ix, step); break;
    }
}

// Per active slot: frames whose parity check has not succeeded by the last
// voted iteration (the fail flags of the vote written in this step).
__global__ __launch_bounds__(kBlock) void engine_status(const SlotDesc *slots, int n, int step,
                                                        int4 *status) {
    const int s = blockIdx.x;
    if (s >= n) return;
    const SlotDesc &S = slots[s];
    const int t = step - S.start_step + 1;          // iteration run in this step
    const int voted = (t == S.T + 1) ? S.T : t - 1;  // iteration whose vote ran in this step
    __shared__ int total;
    if (threadIdx.x == 0) total = voted >= 0 ? 0 : S.F;
    __syncthreads();
    if (voted >= 0)
        for (int f = threadIdx.x; f < S.F; f += kBlock)
            if (S.fail[(size_t)voted * S.F + f] != 0) atomicAdd(&total, 1);
    __syncthreads();
    if (threadIdx.x == 0) status[s] = make_int4(S.slot_id, S.generation, t, total);
}

__global__ void engine_init_fail(int32_t *fail, int F, int T, int early_stop, int check_from) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= (T + 1) * F) return;
    const int t = i / F;
    const bool checked = (t == T) || (early_stop && t >= check_from);
    fail[i] = checked ? 0 : 1;
}

__global__ __launch_bounds__(kBlock) void engine_pack_syndrome(CodeDev c, const uint8_t *syn,
                                                               uint64_t *synbits, size_t frame) {
    pack_syndrome_work(c, syn, synbits, frame, blockIdx.z, blockIdx.y, blockIdx.x);
}

__global__ __launch_bounds__(kBlock) void engine_init_totals(CodeDev c, const float *llr,
                                                             float *tot, size_t frame) {
    init_totals_work(c, llr, tot, frame, blockIdx.z, blockIdx.y, blockIdx.x);
}

__global__ __launch_bounds__(kBlock) void engine_init_psi(CodeDev c, const float *llr, float *psi,
                                                          size_t frame) {
    init_psi_work(c, llr, psi, frame, blockIdx.z, blockIdx.y, blockIdx.x);
}

__global__ __launch_bounds__(64) void engine_frame_exit(FinArgs A) { frame_exit_work(A, blockIdx.x); }

__global__ __launch_bounds__(kBlock) void engine_finalize(CodeDev c, FinArgs A) {
    finalize_work(c, A, blockIdx.z, blockIdx.y, blockIdx.x);
}

inline unsigned tiles_of(int n) { return (unsigned)((n + kBlock - 1) / kBlock); }
inline size_t round_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

}  // namespace

// ------------------------------------------------------------------- arena
void *Arena::alloc(size_t bytes) {
    bytes = round_up(bytes, 256);
    for (Chunk &ch : chunks) {
        for (size_t i = 0; i < ch.free_list.size(); ++i) {
            Range &r = ch.free_list[i];
            if (r.size >= bytes) {
                const size_t off = r.off;
                r.off += bytes;
                r.size -= bytes;
                if (r.size == 0) ch.free_list.erase(ch.free_list.begin() + (long)i);
                return static_cast<char *>(ch.base) + off;
            }
        }
    }
    return nullptr;
}

// A new chunk of at least `at_least` bytes, if the chunks stay within `cap`.
bool Arena::grow(size_t at_least, size_t cap) {
    size_t size = std::max(chunk_bytes, round_up(at_least, 256));
    if (total_bytes + size > cap) size = round_up(at_least, 256);  // a last, smaller chunk
    if (total_bytes + size > cap) return false;
    void *p = nullptr;
    if (hipMalloc(&p, size) != hipSuccess) return false;
    chunks.push_back(Chunk{p, size, {Range{0, size}}});
    total_bytes += size;
    return true;
}

// Return every chunk with no live allocation to the device, after the work
// enqueued on `stream` (read-outs of retired requests) has finished with it.
void Arena::free_idle_chunks(hipStream_t stream) {
    bool synced = false;
    for (size_t i = 0; i < chunks.size();) {
        Chunk &ch = chunks[i];
        if (ch.free_list.size() == 1 && ch.free_list[0].off == 0 && ch.free_list[0].size == ch.size) {
            if (!synced) {
                (void)hipStreamSynchronize(stream);
                synced = true;
            }
            (void)hipFree(ch.base);
            total_bytes -= ch.size;
            chunks.erase(chunks.begin() + (long)i);
        } else {
            ++i;
        }
    }
}

void Arena::release(void *p, size_t bytes) {
    bytes = round_up(bytes, 256);
    for (Chunk &ch : chunks) {
        char *b = static_cast<char *>(ch.base);
        if (p < ch.base || static_cast<char *>(p) >= b + ch.size) continue;
        const size_t off = (size_t)(static_cast<char *>(p) - b);
        auto it = std::lower_bound(ch.free_list.begin(), ch.free_list.end(), off,
                                   [](const Range &r, size_t o) { return r.off < o; });
        it = ch.free_list.insert(it, Range{off, bytes});
        // coalesce with the neighbours
        if (it + 1 != ch.free_list.end() && it->off + it->size == (it + 1)->off) {
            it->size += (it + 1)->size;
            ch.free_list.erase(it + 1);
        }
        if (it != ch.free_list.begin() && (it - 1)->off + (it - 1)->size == it->off) {
            (it - 1)->size += it->size;
            ch.free_list.erase(it);
        }
        return;
    }
}

void Arena::destroy() {
    for (Chunk &ch : chunks) (void)hipFree(ch.base);
    chunks.clear();
    total_bytes = 0;
}

// ------------------------------------------------------------------ engine
hipError_t Engine::init(size_t budget, int slots, bool fp16_, bool early, int cpt_, void *strm) {
    budget_bytes = budget;
    cpt = cpt_;
    max_slots = std::min(slots, kEngineMaxSlots);
    fp16 = fp16_;
    early_stop = early;
    stream = static_cast<hipStream_t>(strm);
    arena.chunk_bytes = std::min<size_t>(budget, (size_t)1 << 30);
    slot.assign(max_slots, Slot{});
    hipError_t e = hipMalloc(&d_slots, sizeof(SlotDesc) * kEngineMaxSlots);
    if (e != hipSuccess) return e;
    e = hipMalloc(&d_status, sizeof(int4) * kEngineMaxSlots);
    if (e != hipSuccess) return e;
    e = hipHostMalloc(&h_table, sizeof(SlotDesc) * kEngineMaxSlots * kStatusRing);
    if (e != hipSuccess) return e;
    e = hipHostMalloc(&h_status, sizeof(int4) * kEngineMaxSlots * kStatusRing);
    if (e != hipSuccess) return e;
    std::memset(h_status, 0, sizeof(int4) * kEngineMaxSlots * kStatusRing);
    for (int i = 0; i < kStatusRing; ++i) {
        if ((e = hipEventCreateWithFlags(&status_ev[i], hipEventDisableTiming)) != hipSuccess) return e;
        if ((e = hipEventCreateWithFlags(&table_ev[i], hipEventDisableTiming)) != hipSuccess) return e;
        status_pending[i] = false;
        table_used[i] = false;
    }
    return hipSuccess;
}

void Engine::destroy() {
    if (stream) (void)hipStreamSynchronize(stream);
    else (void)hipDeviceSynchronize();
    arena.destroy();
    if (d_slots) (void)hipFree(d_slots);
    if (d_status) (void)hipFree(d_status);
    if (h_table) (void)hipHostFree(h_table);
    if (h_status) (void)hipHostFree(h_status);
    for (int i = 0; i < kStatusRing; ++i) {
        if (status_ev[i]) (void)hipEventDestroy(status_ev[i]);
        if (table_ev[i]) (void)hipEventDestroy(table_ev[i]);
    }
    for (const Finishing &fz : finishing) (void)hipEventDestroy(fz.ev);
    for (hipEvent_t ev : spare_events) (void)hipEventDestroy(ev);
}

size_t Engine::request_bytes(const CodeDev &c, int F, int T, bool fp16_) {
    return work_layout(c, F, T, fp16_, false).total;
}

int64_t Engine::submit(const Request &rq) {
    Request r = rq;
    r.ticket = next_ticket++;
    pending.push_back(r);
    return r.ticket;
}

// Edge visits of one iteration of a request: frames x (stored + degree-1
// blocks) x Z.
static int64_t request_edges(const Request &rq) {
    return (int64_t)rq.F * (int64_t)(rq.c.NS + rq.c.ND1) * rq.c.Z;
}

bool Engine::admit_one(const Request &rq, int s) {
    const size_t need = request_bytes(rq.c, rq.F, rq.T, fp16);
    if (in_use + need > budget_bytes) return false;
    const int64_t work = request_edges(rq);
    if (max_step_edges > 0 && active_edges > 0 && active_edges + work > max_step_edges)
        return false;
    void *p = arena.alloc(need);
    if (!p) {
        // the chunks may not outgrow the budget: first return idle chunks
        // (which only frees room when nothing of theirs is in flight)
        if (!arena.grow(need, budget_bytes)) {
            arena.free_idle_chunks(stream);
            p = arena.alloc(need);
            if (!p && !arena.grow(need, budget_bytes)) return false;
        }
        if (!p) p = arena.alloc(need);
        if (!p) return false;
    }
    in_use += need;
    active_edges += work;
    Slot &sl = slot[s];
    sl.active = true;
    sl.all_done = false;
    sl.generation += 1;
    sl.req = rq;
    sl.mem = p;
    sl.mem_bytes = need;
    sl.start_step = step_no;

    SlotDesc &D = sl.desc;
    D = SlotDesc{};
    D.c = rq.c;
    D.L = work_layout(rq.c, rq.F, rq.T, fp16, false);
    char *ws = static_cast<char *>(p);
    D.llr = rq.llr;
    D.msg = ws + D.L.msg;
    D.tot = reinterpret_cast<float *>(ws + D.L.tot);
    D.psi = reinterpret_cast<float *>(ws + D.L.psi);
    D.d1b[0] = reinterpret_cast<uint64_t *>(ws + D.L.d1bits);
    D.d1b[1] = D.d1b[0] + (size_t)rq.F * D.L.d1bits_frame;
    D.synbits = reinterpret_cast<uint64_t *>(ws + D.L.synbits);
    D.fail = reinterpret_cast<int32_t *>(ws + D.L.fail);
    D.part = reinterpret_cast<float *>(ws + D.L.part);
    D.F = rq.F;
    D.T = rq.T;
    D.early_stop = early_stop ? 1 : 0;
    D.check_from = 0;
    D.start_step = step_no;
    D.slot_id = s;
    D.generation = sl.generation;
    D.cn_tiles = (int)check_tiles(rq.c.Z, cpt);
    D.vn_tiles = (int)variable_tiles(rq.c.Z, vn_vpt<float>());
    D.g_tiles = (rq.c.Z + kBlock - 1) / kBlock;

    const CodeDev &c = rq.c;
    const int nfail = (rq.T + 1) * rq.F;
    engine_init_fail<<<dim3((nfail + kBlock - 1) / kBlock), dim3(kBlock), 0, stream>>>(
        D.fail, rq.F, rq.T, D.early_stop, D.check_from);
    engine_pack_syndrome<<<dim3(setup_tiles(c.Z), c.mb, rq.F), dim3(kBlock), 0, stream>>>(
        c, rq.syndrome, D.synbits, D.L.synbits_frame);
    if (c.NC > 0)
        engine_init_totals<<<dim3(setup_tiles(c.Z), c.NC, rq.F), dim3(kBlock), 0, stream>>>(
            c, rq.llr, D.tot, D.L.tot_frame);
    if (c.ND1 > 0)
        engine_init_psi<<<dim3(setup_tiles(c.Z), c.ND1, rq.F), dim3(kBlock), 0, stream>>>(
            c, rq.llr, D.psi, D.L.psi_frame);
    table_dirty = true;
    return true;
}

void Engine::retire(int s) {
    Slot &sl = slot[s];
    const SlotDesc &D = sl.desc;
    FinArgs fa{};
    fa.llr = D.llr;
    fa.tot = D.tot;
    fa.d1bits[0] = D.d1b[0];
    fa.d1bits[1] = D.d1b[1];
    fa.d1post[0] = fa.d1post[1] = nullptr;
    fa.fail = D.fail;
    fa.bits_out = sl.req.bits_out;
    fa.iters_out = sl.req.iters_out;
    fa.conv_out = sl.req.conv_out;
    fa.llr_out = nullptr;
    fa.tot_frame = D.L.tot_frame;
    fa.d1_frame = D.L.d1bits_frame;
    fa.psi_frame = D.L.psi_frame;
    fa.F = D.F;
    fa.T = D.T;
    engine_frame_exit<<<dim3(D.F), dim3(64), 0, stream>>>(fa);
    engine_finalize<<<dim3(tiles_of(D.c.Z), D.c.nb, D.F), dim3(kBlock), 0, stream>>>(D.c, fa);
    hipEvent_t ev = nullptr;
    if (!spare_events.empty()) {
        ev = spare_events.back();
        spare_events.pop_back();
    } else if (hipEventCreateWithFlags(&ev, hipEventDisableTiming) != hipSuccess) {
        ev = nullptr;
    }
    if (ev) (void)hipEventRecord(ev, stream);
    finishing.push_back(Finishing{sl.req.ticket, ev});
    // later kernels on this stream run after the read-out, so the space can be reused now
    arena.release(sl.mem, sl.mem_bytes);
    in_use -= sl.mem_bytes;
    active_edges -= request_edges(sl.req);
    sl.active = false;
    table_dirty = true;
}

hipError_t Engine::step(int *active_out, int *queued_out) {
    // 1. status of earlier steps -> slots whose frames have all stopped
    for (int i = 0; i < kStatusRing; ++i) {
        if (!status_pending[i] || hipEventQuery(status_ev[i]) != hipSuccess) continue;
        status_pending[i] = false;
        const int4 *st = h_status + (size_t)i * kEngineMaxSlots;
        for (int k = 0; k < status_count[i]; ++k) {
            const int s = st[k].x;
            if (s < 0 || s >= max_slots) continue;
            Slot &sl = slot[s];
            if (sl.active && sl.generation == st[k].y && st[k].w == 0) sl.all_done = true;
        }
    }
    // 2. retire finished slots: all frames stopped, or the final vote has run
    for (int s = 0; s < max_slots; ++s) {
        Slot &sl = slot[s];
        if (!sl.active) continue;
        const int last_t = step_no - sl.start_step;  // iterations run before this step
        if (sl.all_done || last_t >= sl.req.T + 1) {
            sl.all_done = false;
            retire(s);
        }
    }
    // 3. admit waiting requests in arrival order while slots and budget allow
    while (!pending.empty()) {
        int s = -1;
        for (int k = 0; k < max_slots; ++k)
            if (!slot[k].active) {
                s = k;
                break;
            }
        if (s < 0 || !admit_one(pending.front(), s)) break;
        pending.pop_front();
    }
    // 4. publish the slot table when it changed
    SlotIndex cn{}, vn{};
    int n = 0, cn_total = 0, vn_total = 0;
    std::vector<int> order;
    for (int s = 0; s < max_slots; ++s)
        if (slot[s].active) order.push_back(s);
    n = (int)order.size();
    if (n > 0) {
        const int ring = table_next;
        if (table_dirty) {
            if (table_used[ring]) (void)hipEventSynchronize(table_ev[ring]);
            SlotDesc *h = h_table + (size_t)ring * kEngineMaxSlots;
            for (int i = 0; i < n; ++i) h[i] = slot[order[i]].desc;
            hipError_t e = hipMemcpyAsync(d_slots, h, sizeof(SlotDesc) * n, hipMemcpyHostToDevice,
                                          stream);
            if (e != hipSuccess) return e;
            (void)hipEventRecord(table_ev[ring], stream);
            table_used[ring] = true;
            table_next = (ring + 1) % kStatusRing;
            table_dirty = false;
        }
        cn.n = vn.n = n;
        for (int i = 0; i < n; ++i) {
            const SlotDesc &D = slot[order[i]].desc;
            cn.begin[i] = cn_total;
            vn.begin[i] = vn_total;
            // this step runs the slot's iteration t; t = T + 1 is its vote-only pass
            const bool vote_only = step_no - D.start_step + 1 == D.T + 1;
            const int gitems = vote_only ? 0 : D.c.n_groups * D.g_tiles;
            const int rows = vote_only ? D.c.mb : D.c.mb - D.c.n_tdom;
            cn.head[i] = SlotHead{D.c.row_desc, D.fail, D.cn_tiles, rows, D.start_step, D.T, D.F, 0,
                                  gitems, D.g_tiles};
            vn.head[i] = SlotHead{D.c.core_tab, D.fail, D.vn_tiles, D.c.NC, D.start_step, D.T, D.F,
                                  D.c.core_tab_stride, 0, 1};
            cn_total += (gitems + D.cn_tiles * rows) * D.F;
            vn_total += D.vn_tiles * D.c.NC * D.F;
        }
        cn.begin[n] = cn_total;
        vn.begin[n] = vn_total;
        int max_deg = 0;  // twice the largest half of a column's terms (the batch width)
        for (int i = 0; i < n; ++i)
            max_deg = std::max(max_deg, 2 * slot[order[i]].desc.c.max_half_terms);
        // 5. one iteration of every active slot, then the status copy
        const dim3 gc(xcd_grid((unsigned)cn_total)), gv(xcd_grid((unsigned)vn_total)), b(kBlock);
        if (fp16) {
            if (cpt == 1) engine_check_pass<_Float16, 1><<<gc, b, 0, stream>>>(d_slots, cn, step_no);
            else if (cpt == 2) engine_check_pass<_Float16, 2><<<gc, b, 0, stream>>>(d_slots, cn, step_no);
            else engine_check_pass<_Float16, 4><<<gc, b, 0, stream>>>(d_slots, cn, step_no);
            if (vn_total > 0) launch_engine_variable<_Float16>(gv, b, stream, d_slots, vn, step_no, max_deg);
        } else {
            if (cpt == 1) engine_check_pass<float, 1><<<gc, b, 0, stream>>>(d_slots, cn, step_no);
            else if (cpt == 2) engine_check_pass<float, 2><<<gc, b, 0, stream>>>(d_slots, cn, step_no);
            else engine_check_pass<float, 4><<<gc, b, 0, stream>>>(d_slots, cn, step_no);
            if (vn_total > 0) launch_engine_variable<float>(gv, b, stream, d_slots, vn, step_no, max_deg);
        }
        const int sr = status_next;
        if (status_pending[sr]) (void)hipEventSynchronize(status_ev[sr]);
        engine_status<<<dim3(n), dim3(kBlock), 0, stream>>>(d_slots, n, step_no, d_status);
        hipError_t e = hipMemcpyAsync(h_status + (size_t)sr * kEngineMaxSlots, d_status,
                                      sizeof(int4) * n, hipMemcpyDeviceToHost, stream);
        if (e != hipSuccess) return e;
        (void)hipEventRecord(status_ev[sr], stream);
        status_pending[sr] = true;
        status_count[sr] = n;
        status_next = (sr + 1) % kStatusRing;
    }
    ++step_no;
    if (active_out) *active_out = n;
    if (queued_out) *queued_out = (int)pending.size();
    return hipGetLastError();
}

int Engine::poll(int64_t *tickets, int cap) {
    int k = 0;
    for (size_t i = 0; i < finishing.size() && k < cap;) {
        const Finishing fz = finishing[i];
        const bool done = fz.ev ? hipEventQuery(fz.ev) == hipSuccess
                                : hipStreamQuery(stream) == hipSuccess;
        if (done) {
            tickets[k++] = fz.ticket;
            if (fz.ev) spare_events.push_back(fz.ev);
            finishing.erase(finishing.begin() + (long)i);
        } else {
            ++i;
        }
    }
    return k;
}

}  // namespace ldpc
