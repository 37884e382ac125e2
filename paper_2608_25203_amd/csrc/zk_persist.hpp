// zk_persist.hpp -- the persistent form of a batch step (declarations shared
// by the kernel unit zk_persist.hip and the batch driver zk_batch.cpp).
//
// One launch runs a whole merged segment of the batch (for example one RK4
// step of every tile).  Its work is a queue of units in phase order; a unit
// is a chunk of consecutive blocks of one tile's row or column pass for one
// program or task.  Workers (blocks of 512 threads, as many as fit the chip)
// take units in queue order from a ticket counter, wait until every unit of
// the same tile's earlier passes has finished (a per-tile completion
// counter), run the unit's blocks with the team shape's row or column body,
// and count the unit as finished.  Every dependency of a unit lies earlier in
// the queue and was taken by a running worker, so each wait ends; a wait is
// still bounded, and one that runs out sets a flag the host reports.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "zk_kernels.hpp"

namespace zk {

struct PUnit {
  int32_t shape;  // persistent shape id (persist_shape)
  int32_t rec;    // argument record: 2 tile + (padded pass ? 0 : 1)
  int32_t index;  // program (row pass) or task (column pass) of that record's schedule
  int32_t blk0;   // first block of the pass this unit runs
  int32_t nblk;   // consecutive blocks it runs
  int32_t tile;   // tile whose completion counter the unit waits on and bumps
  uint32_t need;  // finished units of that tile before this one may start
  int32_t pad_;
};

// Counter words of one launch: [0] ticket, [1] timed-out flag (sticky over
// the launches of one zk_batch_step call), [kCtrDone + t] finished units of
// tile t.
constexpr int kCtrDone = 2;

// Team shapes the persistent kernel hosts, all in blocks of kPBlock threads
// (kPBlock / T teams each): the padded (E = 3) and base (E = 2) transforms
// of 128 to 1024 points per axis; row passes ids 0..7, column passes 8..15,
// with (T, E) in this order.
constexpr int kPBlock = 512;
constexpr int kPShapes = 8;
constexpr int kPShapeT[kPShapes] = {64, 64, 128, 128, 256, 256, 512, 512};
constexpr int kPShapeE[kPShapes] = {3, 2, 3, 2, 3, 2, 3, 2};
// id of (row, T, E), or -1 if the persistent kernel does not host it
inline int persist_shape(bool row, int T, int E) {
  for (int i = 0; i < kPShapes; ++i)
    if (kPShapeT[i] == T && kPShapeE[i] == E) return (row ? 0 : kPShapes) + i;
  return -1;
}
// dynamic LDS bytes a shape needs (BodyLds)
template <typename real>
int persist_lds_bytes(int shape);
template <>
int persist_lds_bytes<double>(int shape);
template <>
int persist_lds_bytes<float>(int shape);

// Zero the ticket and the per-tile counters of a launch (not the flag).
hipError_t launch_persist_reset(uint32_t *ctr, int ntiles, hipStream_t s);
// Clear the timed-out flag.
hipError_t launch_persist_clear_flag(uint32_t *ctr, hipStream_t s);
// The persistent launch: `workers` blocks of kPBlock threads with `lds` bytes of
// dynamic LDS; a dependency wait gives up after spin_limit sleeps.
template <typename real>
hipError_t launch_persistent(int workers, int lds, hipStream_t s, const RowArgs<real> *rargs,
                             const ColArgs<real> *cargs, const PUnit *units, int nunits, uint32_t *ctr,
                             uint32_t spin_limit);
template <>
hipError_t launch_persistent<double>(int, int, hipStream_t, const RowArgs<double> *, const ColArgs<double> *,
                                     const PUnit *, int, uint32_t *, uint32_t);
template <>
hipError_t launch_persistent<float>(int, int, hipStream_t, const RowArgs<float> *, const ColArgs<float> *,
                                    const PUnit *, int, uint32_t *, uint32_t);
// Resident workers per CU with `lds` bytes of dynamic LDS.
template <typename real>
int persistent_blocks_per_cu(int lds);
template <>
int persistent_blocks_per_cu<double>(int lds);
template <>
int persistent_blocks_per_cu<float>(int lds);

}  // namespace zk
