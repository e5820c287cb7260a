// Generic gather-scatter over compressed rows (the "gs" kernel of paper
// Sec. V-B for any id map): device launch and host-side row construction,
// both defined in sem_gs.hip.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace semk {

// In place on w (n doubles): every copy of row r, ids[offsets[r] ..
// offsets[r+1]-1], receives the row's sum, added in row order from 0.  ids
// holds n_copies entries; a row reaching outside them is skipped.
hipError_t launch_gs_rows(int32_t n_rows, const int32_t *offsets, const int32_t *ids,
                          int64_t n_copies, int64_t n, double *w, hipStream_t s);

// Rows of the ids in gid[0..n-1] that occur at least twice (ascending id,
// copies in ascending L index).  Null offsets and ids: sizes only.  Returns
// SEM_OK or an error code with *why set.
int build_gs_csr(int64_t n, const int64_t *gid, int32_t *offsets, int64_t offsets_cap,
                 int32_t *ids, int64_t ids_cap, int32_t *n_rows, int64_t *n_copies,
                 const char **why);

}  // namespace semk
