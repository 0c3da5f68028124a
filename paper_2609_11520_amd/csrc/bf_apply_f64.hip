// F64 instantiation of the butterfly apply kernels.
#include "bf_apply.h"

namespace fio {
void bf_apply_f64(fio_bf_s *bf, bool adj, const double2 *X, long ldx, double2 *Y, long ldy, int nrhs,
                 const cpx<double> *F, void *ws, hipStream_t s, const double2 *Ysub, long ldsub) {
    apply_t<double>(bf, adj, X, ldx, Y, ldy, nrhs, F, ws, s, false, Ysub, ldsub);
}
}  // namespace fio
