// Host-side objects behind the opaque handles of the C ABI: the context
// (library-owned buffers, events, the captured batch graph) and a solver
// state.  Only the ABI implementation uses them; no kernel does.
#pragma once

#include <string>

#include "internal.h"

struct tgv_ctx {
    int device;
    int cus;  // compute units of the device
    std::string err;
    // pinned staging for the camera table and the scans' boundary tables,
    // and its device copy (bytes)
    char *cams_host;
    char *cams_dev;
    long long cams_cap;
    hipEvent_t cams_evt;   // after the upload of the staging buffer
    hipEvent_t cams_done;  // after the last kernel that read cams_dev
    // energy reduction scratch
    double *partials;
    int partials_cap;
    tgv::EnergyOut *eout_dev;
    tgv::EnergyOut *eout_host;
    // state used by tgv_solve when the caller passes none
    tgv_state *own;
    hipEvent_t own_done;  // after the last solve that used it
    // batched solves: block and tile tables, queue counters, captured graph
    tgv::BatchBlock *bt_blocks_dev, *bt_blocks_host;
    int4 *bt_tiles_dev, *bt_tiles_host;
    int bt_blocks_cap, bt_tiles_cap;
    hipEvent_t bt_evt;   // after the upload of the staging tables
    hipEvent_t bt_done;  // after the last launch that read the tables and counters
    int *counters;
    hipGraphExec_t graph_exec;
    std::string graph_key;
    hipStream_t side;
    hipEvent_t ev_a, ev_b;
    // crossing extraction scratch
    void *ext_scratch;
    long long ext_cap;
    unsigned long long *ext_total_host;
    // coarse-to-fine workspace: every level's histograms and u, one state
    void *c2f_mem;
    long long c2f_cap;
    hipEvent_t c2f_done;  // after the last call that used it
};

struct tgv_state {
    tgv_grid grid;
    int storage;
    void *mem;              // one allocation holding every field
    bool owned;             // false: caller-owned memory (tgv_state_wrap)
    long long n;
    float *u[2];
    void *v[2];
    void *p[2];
    void *q[2];
    int xc, yc;             // current primal and dual buffer
    bool fresh;             // previous iterate == current (no step taken yet)
    bool open;              // the last iteration's dual half is done, its primal half pending
    int open_tvl1;          // the model the state was opened with
    int64_t iters_done;
};
