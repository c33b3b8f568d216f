// Internal layout of a simulation handle, shared by the single-lattice and
// batched runtimes.
#pragma once

#include "../../include/lbcg.h"
#include "lbcg_internal.h"

struct lbcg_sim {
    int lattice, prec, collision, kernel;
    int device;             // HIP device current at creation
    int Q, D;
    lbcg::Geo g;
    lbcg::ModelD md;
    lbcg::FusedShape shape;
    size_t elem;            // bytes per stored value
    size_t state_bytes;     // one state buffer
    void *buf[2];
    int cur;                // buffer holding the current state
    bool pulled;            // true: buffer holds post-collision values (pull to read S_t)
    bool initialised;
    int64_t step;
    void *psi;              // generic phase-field scratch (N values of the compute type)
    void *moms;             // split geometry step: its scratch (split_scratch_bytes), or null
    lbcg::SplitPlan split;  // its block list lengths
    double *partials, *diag;
    uint32_t *ctr;          // time-step counter pair: ctr[cur] = steps taken since initialisation
    double *staging;        // field / population staging
    int64_t staging_nodes;
    uint8_t *mask_dev;
    lbcg::DevInlet *in_dev;
    lbcg::DevOutlet *out_dev;
    hipStream_t stream;         // where the handle's work is queued
    hipStream_t owned_stream;   // the stream the library created for it, or null
    void *arena;
    bool own_arena;
    size_t arena_bytes;
    // Compact state (LBCG_KERNEL_COMPACT): cbuf[cur] holds the state while
    // compact is true; before a read of the state it is expanded into buf[cur]
    // (expanded marks that buf[cur] is current).
    void *cbuf[2];
    bool compact, expanded;
    hipGraphExec_t graph[2];  // graph_steps steps starting from buffer 0 / 1
    int graph_steps;
    bool graph_failed;
};

