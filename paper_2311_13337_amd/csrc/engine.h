// engine.h -- device data layout and kernel launchers of the sweep engine
// (internal to libvadx; the public boundary is include/vadx.h).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "adex_model.h"

namespace vadx {

// Largest number of steps integrated between two synchronisations of the
// waves of an instance (one block). A block of B steps reads the delay rings
// before writing any of its own rates, which is exact as long as
// B <= d_min + 1 (the shortest delay plus one).
constexpr int kMaxBlock = 32;
// With wave slack a block is at most (d_min + 1) / 2 steps, so the waves of an
// instance may drift at least a block apart; taken only where such a block is
// still this long.
constexpr int kSlackMinBlock = 12;

// One instance = one parameter combination on one connectome.
struct InstDev {
    float S, be, ae;
    float w_noise, inv_tauw_e;  // noise weight, 1/tau_w of the excitatory population
    float cF[4];                // external drives c_F: ee, ei, ie, ii
    int32_t n;          // regions
    int32_t D;          // ring depth in steps
    int32_t conn;       // connectome
    uint32_t id;        // instance index (Philox key word 1)
    int32_t Dp;         // ring row stride: D + B - 1 (mirror of the first B - 1 slots)
    int64_t table_off;  // into the packed delay tables (nnz entries)
    int64_t trace_off;  // floats: [n_trace][8][n]; -1: not traced
    int64_t state_off;  // floats (8-byte aligned): [8][n] doubles, final/resume state
    int64_t acc_off;    // floats: [n] running time-average sums
    int64_t ring_off;   // floats: [n][Dp] excitatory-rate history
    int64_t samp_off;   // floats: [n_samples][n]
    int64_t fc_off;     // floats: [n][n]
};

// Connectome in CSR form (ascending column order inside each row).
struct ConnDev {
    int32_t n, nnz;
    int64_t row_off;    // into rowptr (n + 1 entries)
    int64_t edge_off;   // into colw / len arrays (nnz entries)
    int64_t sc_off;     // into raw weights (n*n doubles)
    int64_t ref_off;    // into reference FC matrices (n*n floats); -1: none
};

// A workgroup's share: `count` instances of the same region count and block
// length, on consecutive lanes (instance s on lanes [s n, (s + 1) n)).
struct GroupDev {
    int32_t first;      // into the instance permutation
    int32_t count;
    int32_t n;
    int32_t block;      // steps per block (<= d_min + 1 of every instance)
    int32_t dmin;       // shortest delay in steps over the group's instances
};

struct DelayTableDev {
    int32_t conn;
    float v;            // conduction speed (m/s)
    int64_t off;        // into packed edges: (column << 20) | delay
};

struct IntegrateArgs {
    KModel M;
    const KModel *Mp;           // the same constants in device memory (read per queue item)
    const InstDev *inst;
    const int32_t *perm;
    const GroupDev *groups;
    const ConnDev *conns;
    const int32_t *rowptr;
    const float *weight;        // row-normalised weights per CSR edge
    const int32_t *packed;      // per delay table and edge: (column << 20) | delay
    float *ws;                  // workspace base (floats)
    uint32_t *flags;            // per instance
    int64_t n_steps_total, transient_steps, tavg_steps, n_trace_steps, n_samples;
    int64_t n_begin, n_end;
    double dt, gdw_scale;       // gdw_scale = sigma_OU / tau_OU * sqrt(dt) (0: noise off)
    double E_init, I_init;
    uint32_t seed;
    int32_t integrator;
    int32_t block;              // one workgroup per group: the groups' block length;
                                // persistent: the longest block length (sizes the LDS)
    uint32_t *status;           // bit 1: a wait for another wave's block timed out
    uint32_t wait_spins;        // bound of that wait
};

// Work queue of the persistent integration kernel (in the workspace).
struct QueueArgs {
    int *next;                  // next item to hand out
    int *done;                  // per group: chunks completed in this launch
    uint32_t *status;           // bit 0: a wait for a previous chunk timed out
    int n_groups, n_items;
    int64_t item_steps;
    uint32_t max_spins;
};

struct FcArgs {
    const InstDev *inst;
    const ConnDev *conns;
    const double *sc;           // raw weights, [n][n] per connectome
    const float *ref;           // reference FC matrices, [n][n] per connectome that has one
    float *ws;
    float *stats;               // [inst][8] as vadx_stats (6 floats + flags + fc_fit)
    uint32_t *flags;
    int64_t n_samples;
    double min_var;             // silence threshold on a region's variance
    int32_t max_n;              // most regions of an instance (sizes the LDS)
};

// Launchers (return hipError_t of the launch).
hipError_t launch_conn_prepare(int n, const double *w, const double *len, int32_t *rowptr,
                               float *weight, double *edge_len, int32_t *colidx, hipStream_t s);
hipError_t launch_delays(int n_tables, const DelayTableDev *tables, const ConnDev *conns,
                         const int32_t *colidx, const double *edge_len, double dt,
                         int32_t *packed, int max_nnz, hipStream_t s);
hipError_t launch_fill_u32(uint32_t *p, int64_t n, uint32_t value, hipStream_t s);
// Copies m to device memory (out) on stream s.
hipError_t launch_kmodel_store(const KModel &m, KModel *out, hipStream_t s);
// One workgroup per group (all of block length a.block) over [a.n_begin, a.n_end).
hipError_t launch_integrate(const IntegrateArgs &a, int n_groups, int block_threads, hipStream_t s);
// The persistent kernel: `grid` workgroups drain the queue of (group, chunk)
// items over a.groups (any block lengths up to a.block); occ: waves per SIMD
// of its register budget (2 or 3).
hipError_t launch_integrate_persistent(const IntegrateArgs &a, int block_threads, const QueueArgs &q,
                                       int grid, int occ, hipStream_t s);
int persistent_blocks_per_cu(int max_block, int block_threads, int occ);
hipError_t launch_rank_sort(const float *val, const int64_t *idx, int32_t k, int64_t *idx_out,
                            float *val_out, hipStream_t s);
hipError_t launch_fc_stats(const FcArgs &a, int64_t n_inst, hipStream_t s);

} // namespace vadx
