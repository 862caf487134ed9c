// Host-side state of the multi-request engine (engine.hip); internal.
#pragma once

#include "internal.h"

#include <deque>
#include <vector>

namespace ldpc {

constexpr int kEngineMaxSlots = 64;

// Device-resident description of one admitted request (one slot).
struct SlotDesc {
    CodeDev c;
    WorkLayout L;
    const float *llr;
    void *msg;
    float *tot;
    float *psi;
    uint64_t *d1b[2];
    uint64_t *synbits;
    int32_t *fail;
    float *part;             // owner-group partial sums
    int F, T, early_stop, check_from;
    int start_step;          // engine step that runs this slot's iteration 1
    int slot_id, generation;
    int cn_tiles, vn_tiles;  // check-pass and variable-pass tiles per row / column
    int g_tiles;             // check-pass tiles (256 positions) per owner group
};

struct Request {
    CodeDev c;
    int F, T;
    const float *llr;
    const uint8_t *syndrome;
    uint8_t *bits_out;
    int32_t *iters_out;
    uint8_t *conv_out;
    int64_t ticket;
};

// Device memory in 1 GiB chunks (or the budget if smaller), allocated on
// first need; first-fit sub-allocation.  The chunks together never exceed
// the engine's budget: a request that fits the budget but no free range
// waits, and chunks left entirely free are returned to the device when a
// larger request needs the room.
struct Arena {
    struct Range {
        size_t off, size;
    };
    struct Chunk {
        void *base;
        size_t size;
        std::vector<Range> free_list;  // sorted by offset
    };
    size_t chunk_bytes = 0;
    size_t total_bytes = 0;  // device bytes held in chunks
    std::vector<Chunk> chunks;
    void *alloc(size_t bytes);
    bool grow(size_t at_least, size_t cap);
    void release(void *p, size_t bytes);
    void free_idle_chunks(hipStream_t stream);
    void destroy();
};

struct Engine {
    struct Slot {
        bool active = false;
        bool all_done = false;
        int generation = 0;
        int start_step = 0;
        Request req{};
        void *mem = nullptr;
        size_t mem_bytes = 0;
        SlotDesc desc{};
    };
    struct Finishing {
        int64_t ticket;
        hipEvent_t ev;
    };

    size_t budget_bytes = 0, in_use = 0;
    int64_t max_step_edges = 0, active_edges = 0;  // latency cap on the work of one step
    int max_slots = 0;
    bool fp16 = false, early_stop = true;
    int cpt = 4;  // checks per thread of the check kernel (1, 2, 4)
    hipStream_t stream = nullptr;
    int device = 0;
    int step_no = 1;
    int64_t next_ticket = 1;
    Arena arena;
    std::vector<Slot> slot;
    std::deque<Request> pending;
    std::vector<Finishing> finishing;
    std::vector<hipEvent_t> spare_events;
    SlotDesc *d_slots = nullptr;
    int4 *d_status = nullptr;
    SlotDesc *h_table = nullptr;   // pinned, ring of tables
    int4 *h_status = nullptr;      // pinned, ring of status copies
    hipEvent_t status_ev[4] = {};
    hipEvent_t table_ev[4] = {};
    bool status_pending[4] = {};
    bool table_used[4] = {};
    int status_count[4] = {};
    int status_next = 0, table_next = 0;
    bool table_dirty = false;

    hipError_t init(size_t budget, int slots, bool fp16, bool early_stop, int cpt, void *stream);
    void destroy();
    static size_t request_bytes(const CodeDev &c, int F, int T, bool fp16);
    int64_t submit(const Request &r);
    hipError_t step(int *active_out, int *queued_out);
    int poll(int64_t *tickets, int cap);

  private:
    bool admit_one(const Request &r, int s);
    void retire(int s);
};

}  // namespace ldpc
