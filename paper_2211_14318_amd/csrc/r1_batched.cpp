// Uneven batches (placeholder until the persistent scheduler lands).
#include "r1_handle.hpp"

void r1h::release_batched(r1_handle h) { (void)h; }

extern "C" r1_status r1_envelope_batched(r1_handle h, const r1_material* mat,
                                         const r1_lamination* table, int32_t n_table, int64_t n,
                                         const int32_t* lam_idx, r1_dtype dtype, const void* F,
                                         const void* beta_n, void* W, void* P, r1_laminate* tree,
                                         int32_t* flags, void* stream) {
  (void)h; (void)mat; (void)table; (void)n_table; (void)n; (void)lam_idx; (void)dtype; (void)F;
  (void)beta_n; (void)W; (void)P; (void)tree; (void)flags; (void)stream;
  return R1_EUNSUPPORTED;
}
