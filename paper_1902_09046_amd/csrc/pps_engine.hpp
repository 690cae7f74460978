// Epoch engine: runs batches of job rows (and the finalisation of ABC jobs)
// as one captured hipGraph launch per epoch.  A slot owns mapped pinned host
// tables (written by the host before each epoch, copied in by the stage-in
// kernel), device tables, result areas written back by the stage-out kernel,
// and the instantiated graphs of the epoch forms it has run.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <map>
#include <vector>

#include "pps_internal.hpp"
#include "pps_launch.hpp"

namespace pps {

// Rows and finalisations of one epoch.  For each row the caller sets every
// field except tile_size and tile_begin; n_tiles and tile_offset select the
// row's tiles (whole job: tile_offset 0, n_tiles = tiles_for(cls, n)).
struct EpochPlan {
    std::vector<JobDev> rows[N_CLASSES];
    std::vector<FinJob> fins;  // block_begin / n_blocks are set by the engine
    void clear()
    {
        for (auto &r : rows)
            r.clear();
        fins.clear();
    }
};

class EpochEngine {
  public:
    EpochEngine() = default;
    ~EpochEngine();
    EpochEngine(const EpochEngine &) = delete;
    EpochEngine &operator=(const EpochEngine &) = delete;

    // Allocates n_slots staging slots on the current device.
    int init(int n_slots, int cu_count);

    void set_shape(int cls, const SimShape &sh) { shape_.sim[cls] = sh; }
    const SimShape &shape(int cls) const { return shape_.sim[cls]; }
    // Draws per tile: one per workgroup for the cell class, else one per lane
    // and interleaved draw.
    uint64_t tile_size(int cls) const
    {
        if (cls == CLASS_CELLS || cls == CLASS_GILLESPIE)
            return 1;
        return static_cast<uint64_t>(shape_.sim[cls].block) * shape_.sim[cls].dpl;
    }
    uint64_t tiles_for(int cls, uint64_t n) const
    {
        return (n + tile_size(cls) - 1) / tile_size(cls);
    }

    // Stages `plan` into `slot` and launches the epoch graph on `stream`.
    // The slot must be idle (see wait / ready).  When the previous epoch was
    // launched on another stream, this one starts after that epoch's
    // simulation kernels have ended (a job's tiles can span both epochs and
    // its finalisation reads all of them); its finalisation and stage-out
    // still overlap this epoch.
    // With build == false the epoch replays an instantiated graph of its form
    // and launch shape or fails with PPS_EINVAL: nothing is captured,
    // instantiated or destroyed.
    int launch(int slot, EpochPlan &plan, hipStream_t stream, bool build = true);
    // The stream of a slot: `primary` for slot 0, a stream of the engine for
    // the others (so that epochs alternate between two streams).
    hipStream_t slot_stream(int slot, hipStream_t primary) const
    {
        return slot == 0 ? primary : slots_[slot].own_stream;
    }
    // Blocks until the slot's epoch has finished.
    int wait(int slot);
    // Non-blocking: PPS_OK when the slot has no epoch in flight (the last one
    // finished), PPS_PENDING while it runs, or an error status.
    int poll(int slot);
    bool in_flight(int slot) const { return slots_[slot].in_flight; }

    const FinResult *out_fin(int slot) const { return slots_[slot].h_out_fin; }
    const unsigned long long *out_counts(int slot) const { return slots_[slot].h_out_counts; }
    // Duration of the simulation kernels of the slot's last finished epoch.
    float sim_ms(int slot) const { return slots_[slot].sim_ms; }
    // Duration of that epoch's ABC finalisation (selection, compaction,
    // moments), or a negative value if it had none.
    float fin_ms(int slot) const { return slots_[slot].fin_ms; }
    int n_slots() const { return static_cast<int>(slots_.size()); }

  private:
    struct Slot {
        EpochHeader *h_hdr = nullptr;
        JobDev *h_rows = nullptr;
        FinJob *h_fins = nullptr;
        FinResult *h_out_fin = nullptr;
        unsigned long long *h_out_counts = nullptr;
        EpochDevPtrs dev;
        // one graph per epoch form: the classes with tiles (a bit each) and
        // the finalisation (none / with the selection passes / fixed
        // tolerance only), built on first use for the current shape
        std::map<unsigned, hipGraphExec_t> execs;
        bool have_shape = false;
        EpochShape exec_shape;
        hipEvent_t sim_start = nullptr, sim_stop = nullptr, fin_stop = nullptr, done = nullptr;
        hipStream_t own_stream = nullptr;  // slots after the first
        bool in_flight = false;
        bool has_fin = false;  // the epoch in flight has a finalisation
        float sim_ms = -1.0f, fin_ms = -1.0f;
    };
    int set_graph_shape(Slot &s, bool build);
    int graph_for(Slot &s, unsigned form, hipGraphExec_t *out, bool build);
    int finish(Slot &s);

    std::vector<Slot> slots_;
    EpochShape shape_;
    int cu_count_ = 0;
    hipStream_t capture_stream_ = nullptr;
    int last_slot_ = -1;  // slot and stream of the last launched epoch
    hipStream_t last_stream_ = nullptr;
};

}  // namespace pps
