// Persistent batched kernel (batch_persistent.hip): the per-block pipeline
// of a batch (Gram sweep -> k x k step -> update sweep -> ... , Sec. 4.1's
// many independent per-node blocks through Sec. 4.2's passes) as ONE launch.
//
// Workgroups stay resident and take tasks: a task is one workgroup's share
// of one sweep of one block (the same share a workgroup of the launch per
// phase gets, described by the same segment tables).  Opened sweeps sit in
// a queue (first the blocks' Gram sweeps, larger blocks first); a workgroup
// takes a share of the oldest opened sweep that has one left.  The
// workgroup that finishes the last share of a block's sweep reduces that
// sweep's partial sums and runs the block's k x k step itself, then appends
// the block's next sweep to the queue; so the sweeps of different blocks run
// side by side (the DD Gram of one block next to the update of another) and
// no block waits for the slowest block of its phase.  Nothing waits on
// another workgroup: a workgroup that finds no open task pauses briefly and
// retries a bounded number of times, then leaves; the workgroup that opens a
// sweep always goes on to take its tasks, so every opened sweep is finished.
#pragma once
#include "internal.hpp"

namespace borth {

struct PSweep {
  int kind;          // 0: DMA-staged DD Gram, 1: tile DD Gram (256 threads), 2: update
  int K, KYP, GR;    // update class
  int nw;            // update: streaming waves that fit the LDS pool
  int ntasks;        // workgroup shares of the block in this sweep
  int wg0;           // the block's first workgroup index in the sweep's grid
  const void* tab;   // segment table of the sweep (GramSeg or UpdDev)
  const int* map;    // workgroup -> segment
};

struct PBlock {
  int nsweeps;          // 1 + passes
  int pad;
  PSweep sw[3];
  ReduceSeg red[2];     // the reduction of sweep s's partials
  int red_dd[2];
  FactorArgs fac[2];    // the k x k step after sweep s
  int fac_ns[2];        // 16 x 16 threads, NS x NS elements each (k <= 16 NS)
};

// Dynamic LDS of a persistent workgroup (two are resident per compute unit).
constexpr size_t kPersistLds = 80 * 1024;
// Global working memory of one workgroup's k x k step (doubles).
constexpr int64_t kPersistFactorDoubles = 17152;

// Update classes the persistent kernel carries (16 x 16 threads): widths 8,
// 16, 32, 64; (KYP, GR) in {(16, 2), (16, 0), (0, 1), (0, 0)}.
bool persist_update_ok(int K, int KYP, int GR);
// Streaming waves of an update class within the LDS pool (0: does not fit).
int persist_update_waves(int K, int KYP, int GR);
// Resident persistent workgroups on the current device.
int batch_persistent_grid();
// Ints of the launch's state (queue and counters, set by the launch).
int batch_persistent_state_ints(int nb);
// order: blocks by decreasing work; state: batch_persistent_state_ints(nb)
// ints; scratch: grid x kPersistFactorDoubles.  Two launches: the state's
// initialization, then the persistent kernel.
hipError_t launch_batch_persistent(const PBlock* blocks, const int* order, int nb, int* state,
                                   double* scratch, int grid, hipStream_t st);

}  // namespace borth
