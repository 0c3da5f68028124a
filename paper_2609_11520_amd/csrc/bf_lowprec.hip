// Split-FP16 butterfly apply (MFMA with FP32 accumulation).  Not built yet:
// requesting FIO_PREC_SPLIT_FP16 reports FIO_ERR_UNSUPPORTED.
#include "bf.h"

namespace fio {

void bf_make_lowprec(fio_bf_s *, hipStream_t) { throw Err{FIO_ERR_UNSUPPORTED}; }

size_t bf_ws_bytes_split16(const fio_bf_s *, int) { return 0; }

void bf_apply_split16(fio_bf_s *, bool, const double2 *, long, double2 *, long, int, void *, hipStream_t) {
    throw Err{FIO_ERR_UNSUPPORTED};
}

}  // namespace fio
