// Internal interface between the C ABI (prhip.hip) and the batch-update
// kernels (apply.hip).
#pragma once
#include <hip/hip_runtime.h>

// One CSR view of G^{t-1} (n rows, offsets off[n+1], m_old entries cols) updated
// by the deletions (del_row[i], del_col[i]) and insertions, all device
// arrays, into new_off[n+1] / new_cols[m_new]. Enqueued on s and waited for.
// Returns a hipError_t (0 = success); *err_out receives the batch error bits
// (1 ID out of range, 2 repeated pair, 4 deletion absent, 8 insertion
// present, 16 edge count or degree inconsistent, 32 a write outside its row;
// 0 = valid) and *what names a failed runtime step.
int prhip_apply_view(int n, const int *off, const int *cols, int m_old, int m_new, const int *del_row,
                     const int *del_col, int nd, const int *ins_row, const int *ins_col, int ni,
                     int *new_off, int *new_cols, hipStream_t s, int *err_out, const char **what);
