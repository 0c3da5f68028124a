// F32 instantiation of the butterfly apply kernels.
#include "bf_apply.h"

namespace fio {
void bf_apply_f32(fio_bf_s *bf, bool adj, const double2 *X, long ldx, double2 *Y, long ldy, int nrhs,
                 const cpx<float> *F, void *ws, hipStream_t s, bool split) {
    apply_t<float>(bf, adj, X, ldx, Y, ldy, nrhs, F, ws, s, split);
}
}  // namespace fio
