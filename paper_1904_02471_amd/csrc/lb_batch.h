// lb_batch.h -- batched time step over many independent simulations (the
// serving form): one launch advances every admitted simulation by one step.
#pragma once

#include "lb_internal.h"

namespace lbm {

// Device descriptor of one admitted simulation.  `p` is built by the same
// host code as for a single simulation, so a simulation computes the same
// rounded values alone and in a batch.
struct BatchSlot {
    Params<float> p;
    float *buf[3];        // CS: ping-pong pair; FD: g, A, B
    double *partial;      // fused-diagnostics partials of this simulation
    double *series;       // [samples][kDiag] raw sums
    const float *ax, *ay, *bx, *by;  // probe (NULL when unset)
    int model;            // 0: collision-streaming, 1: finite-difference
    int start_epoch;      // batch step at which the simulation was admitted
    int nsteps;           // steps to run
    int every;            // sampling period (>= 1)
    int diag_blocks;      // partials written by one fused step
    int tiles_x;          // FD: tiles per row
};

// One workgroup of a batched launch: simulation `slot`, row (CS) or tile
// (FD) `local`.  FD tiles are 64 x 32 nodes in the first Runge-Kutta stage
// (the canonical tiles of the fused diagnostics) and 64 x 16 or 64 x 32 in
// the later stages (a tuning choice per equilibrium order); a stage's
// output does not depend on the tile shape.
struct BatchWork {
    int slot, local;
};

// The batch step ("epoch") is read from device memory (*epoch), so that a
// captured launch sequence replays unchanged from step to step; a
// simulation steps in a launch while 0 <= epoch - start_epoch < nsteps, and
// its own step index selects the ping-pong buffers and whether the input
// state is sampled.  launch_epoch_advance adds one to *epoch after the
// launches of a step.
hipError_t launch_cs_batch(const BatchSlot *slots, const BatchWork *work, int nwork, const int *epoch,
                           hipStream_t s);
// stage 1 on 64 x 32 tiles; stages 2 and 3 on 64 x (4 rows) tiles, rows 4 or 8
hipError_t launch_fd_batch(const BatchSlot *slots, const BatchWork *work, int nwork, int N, int stage, int rows,
                           const int *epoch, hipStream_t s);
// Sums the partials of every listed simulation that sampled in this epoch
// into its series.
hipError_t launch_finalize_batch(const BatchSlot *slots, const int *slot_ids, int nslots, const int *epoch,
                                 hipStream_t s);
hipError_t launch_epoch_advance(int *epoch, hipStream_t s);

}  // namespace lbm
