// fk_host.hpp -- host-side plan object and helpers shared by the runtime
// translation units (fused path, unfused baseline, cost model, server).
#pragma once
#include <hip/hip_runtime.h>

#include <vector>

#include "../../include/fk.h"
#include "fk_chain.hpp"
#include "fk_internal.hpp"

struct fk_plan {
    static constexpr int kRing = 4;  // item tables in flight
    struct Slot {
        void *h_stage = nullptr;      // pinned host staging of the run table
        void *h_dev = nullptr;        // the staging buffer's device address
        void *d_table = nullptr;      // device run table
        hipEvent_t done = nullptr;    // recorded after the slot's last launch
        bool used = false;
        hipGraphExec_t gexec = nullptr;
        fk_launch_config gcfg = {0, 0};
    };

    fk_chain_desc chain{};                 // ops point into op_descs
    std::vector<fk_op_desc> op_descs;
    int32_t max_batch = 0;
    fk_plan_opts opts{};
    fk_launch_config cfg{};
    int family = 0;                        // fk::FAM_*
    int static_n = 0;                      // compile-time chain length
    std::vector<fk::OpRec> ops;            // normalised run-time op list
    int32_t swap = 0;                      // net channel swap (run-time tier)
    void *d_ops = nullptr;
    void *d_consts = nullptr;
    fk::StatPartial *d_st_part = nullptr;  // stats write: block partials
    uint32_t st_capacity = 0;              // stats write: partial slots held
    size_t table_bytes = 0;
    Slot slots[kRing];
    int next_slot = 0;
    hipStream_t capture_stream = nullptr;
    hipStream_t tune_stream = nullptr;
    int device = 0;
    int num_cus = 256;
};

namespace fk {

fk_status set_error(fk_status s, const char *fmt, ...);
fk_status hip_error(hipError_t e, const char *what);
int dtype_size(int32_t dt);
fk_status validate_chain(const fk_chain_desc *ch);
fk_status validate_items(const fk_chain_desc *ch, const fk_item *items, int32_t n);
bool config_valid(const fk_launch_config &c);
bool per_pixel(const fk_plan *p);
// the plan's kernel runs the run-time op list (not a compile-time chain)
bool runs_op_list(const fk_plan *p);
// The plan's kernel for a launch configuration; `large`: the launch covers
// at least kStridedMinPixels output pixels.
const void *plan_kernel(const fk_plan *p, const fk_launch_config &cfg, bool large = true);
size_t lds_bytes(const fk_plan *p, const fk_launch_config &cfg);
uint32_t build_items(const fk_plan *p, const fk_item *items, int32_t n, const fk_launch_config &cfg,
                     ItemRec *recs, uint32_t *tb, int32_t batch_n = 0);
uint32_t build_table(const fk_plan *p, const fk_item *items, int32_t n, const fk_launch_config &cfg,
                     void *stage);
KArgs make_args(const fk_plan *p, void *d_table);
uint32_t persistent_grid(const fk_plan *p, const fk_launch_config &cfg);
fk_status launch_args(const fk_plan *p, const fk_launch_config &cfg, KArgs &a, uint32_t grid, int32_t n_items,
                      hipStream_t stream, hipEvent_t ev0 = nullptr, hipEvent_t ev1 = nullptr);
fk_status launch(const fk_plan *p, const fk_launch_config &cfg, void *d_table, uint32_t grid,
                 int32_t n_items, hipStream_t stream, hipEvent_t ev0 = nullptr,
                 hipEvent_t ev1 = nullptr);
bool compact_batch(const fk_plan *p, const fk_item *items, int32_t n);
const void *kernel_table_upload();  // fk_table.hip
fk_status run_fused(fk_plan *p, const fk_item *items, int32_t n, const fk_launch_config &cfg,
                    bool graph, hipStream_t stream, hipEvent_t ev0 = nullptr, hipEvent_t ev1 = nullptr);

}  // namespace fk
