// Ensemble engine: many independent lattices stepped by one persistent
// launch per time step.  Shared by the engine kernels and the host side.
#pragma once

#include <hip/hip_runtime.h>

#include "kernels.hpp"

namespace d2q37 {

// One lattice of the ensemble, as the step kernel reads it.  The lattice
// keeps its single-lattice layout (element (l, X, y) at l pstride +
// X cstride + y, 3 unused halo columns per side); the engine wraps x
// instead of refreshing halos.
struct SlotDesc {
  char* buf[2];
  long long pstride;  // elements between populations of a site
  long long cstride;  // elements between columns
  int storage;      // STORAGE_F64 or STORAGE_F32
  int lx, ly;       // lattice size
  int ny_waves;     // wavefront tiles per column: ceil(ly / 64)
  int cur;          // buffer holding the current populations
  int steps_left;   // steps still to run; 0 = finished (not stepped)
  int pad;
  CollideParams cp;
  WallParams wp;
};

// Active-slot table in device memory (ints), one per storage type: [0]
// number of active slots n,
// [1] total tiles, [2, 2 + max_slots) slot ids in tile order,
// [2 + max_slots, 2 + 2 max_slots + 1) first tile of each active slot
// (prefix sums, entry n = total).
inline size_t engine_table_ints(int max_slots) { return 2 + 2 * static_cast<size_t>(max_slots) + 1; }

enum EngineSchedule : int { SCHED_CHUNKED = 0, SCHED_STRIDED = 1 };

// The step kernel of one storage type walks that type's table (arguments
// slots, table, max_slots); the advance kernel covers every slot
// (arguments slots, max_slots, status).
hipError_t launch_engine_step(int storage, const SlotDesc* slots, const int* table, int max_slots,
                              int block, int groups, int schedule, hipStream_t s);
hipError_t launch_engine_advance(SlotDesc* slots, int max_slots, int* status, hipStream_t s);
// Kernel node parameters for a hand-built graph of one engine step.
hipError_t engine_step_node(int storage, int block, int groups, int schedule, void** func, dim3* grid,
                            dim3* threads);
hipError_t engine_advance_node(int max_slots, void** func, dim3* grid, dim3* threads);

}  // namespace d2q37
