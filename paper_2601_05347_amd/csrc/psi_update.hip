// Batch insert and delete (Alg. 4, Sec. 4.2).
#include "psi_index.h"

namespace psi {

psi_status do_insert(psi_index ix, const uint32_t* d_pts, uint64_t m, uint32_t* d_new_ids) {
    (void)ix; (void)d_pts; (void)m; (void)d_new_ids;
    return PSI_E_STATE;
}

psi_status do_delete(psi_index ix, const uint32_t* d_ids, uint64_t m, uint64_t* d_ndeleted) {
    (void)ix; (void)d_ids; (void)m; (void)d_ndeleted;
    return PSI_E_STATE;
}

}  // namespace psi
