// Butterfly factorization handle (Section 2.2) shared by the BF, HSS and solve units.
#pragma once
#include <map>

#include "common.h"

namespace fio {
// Tile configuration of the applies for one (direction, precision, column bucket); 0 = the
// built-in default.  kc: 2D column chunk (8 or 16); nsplit: 2D reduction split of the U / V^*
// steps; kmax: 1D levels per fused pass.
struct TileCfg {
    int kc = 0, nsplit = 0, kmax = 0;
    int leaf_sep = 0;   // 1D: run the first leaf factor as its own kernel (no fold into the first pass)
    int valu = 0;       // 1D split FP16: run the transfer passes as FP32 structured passes (vector units)
};
// Section 5.1's Gaussian-sum amplitude (m = 0: a = 1), passed to the factor generation by value
constexpr int kMaxAmpTerms = 16;
struct Amp {
    int m = 0;
    double s2 = 1.0;
    double x[kMaxAmpTerms] = {}, xi[kMaxAmpTerms] = {};
};
}  // namespace fio

struct fio_bf_s {
    fio_bf_desc desc;
    int dim = 1;
    long N = 0;                        // vector length (n in 1D, n^2 in 2D)
    long n1 = 0;                       // points per dimension
    int L = 0, h = 0, Lp = 0, nl = 0, q = 0, b = 0, nsl = 0;
    int lc = 0, hb = 0;                // 2D: coarse level L - h, log2 of the leaf box width
    // element offsets (complex entries) of each factor inside the packed arrays
    size_t offV = 0, offM = 0, offU = 0, total = 0;
    std::vector<size_t> offC, offB;   // offC[lev] = C^[h+1+lev], offB[lev] = B^[h+1+lev]
    fio::DevBuf f64;                   // complex128 factors, import/export layout
    fio::DevBuf f32;                   // complex64 copy (FIO_PREC_FP32)
    fio::DevBuf f16;                   // split-fp16 transfer blocks: hi and lo planes (FIO_PREC_SPLIT_FP16)
    bool split16 = false;              // FIO_PREC_SPLIT_FP16 copies built (1D, q = 9)
    // structured transfer factors (built on the GPU only): twiddles of every B and C level and
    // the two shared Lagrange matrices P_c(i, t) (host copy, passed as kernel arguments)
    bool structured = false;
    fio::DevBuf tw64, tw32;
    double Pchild[2 * 16 * 16] = {};
    fio::DevBuf adj64, adj32;          // 2D: conjugate-transposed factor copies read by the adjoint
    fio::Amp amp;                      // amplitude of the kernel (copied from the descriptor)
    fio::DevBuf ws;                    // handle-owned workspace (ws == NULL in the applies)
    std::mutex ws_mu;
    std::map<int, fio::TileCfg> tuned; // fio_bf_autotune results, key tile_key(adj, prec, nrhs)
    mutable std::mutex tune_mu;
};

namespace fio {
// Computes the geometry of `d` into `bf` (no allocation).  Returns FIO_OK or FIO_ERR_ARG/UNSUPPORTED.
fio_status bf_plan(const fio_bf_desc *d, fio_bf_s *bf);
size_t bf_coef_elems(const fio_bf_s *bf, int nrhs);   // complex entries of one coefficient buffer
// Internal apply used by the HSS construction and the solver (workspace given explicitly).
// freq_internal (2D only): frequency-side vectors are in the library's Morton order instead of
// the user's lexicographic order (the order of the HSS tree over frequencies).
void bf_apply_impl(fio_bf_s *bf, bool adjoint, const double2 *X, long ldx, double2 *Y, long ldy, int nrhs,
                   fio_prec prec, void *ws, hipStream_t s, bool freq_internal = false);
// R = U - K~ X (FP64) in one pass where the leaf kernel can subtract (1D); false otherwise
bool bf_residual_f64(fio_bf_s *bf, const double2 *X, long ldx, const double2 *U, long ldu, double2 *R, long ldr,
                     int nrhs, void *ws, hipStream_t s);
// 2D butterflies (bf2d.hip)
fio_status bf2d_plan(const fio_bf_desc *d, fio_bf_s *bf);
size_t bf2d_ws_bytes(const fio_bf_s *bf, int nrhs, fio_prec prec);
void bf2d_generate(fio_bf_s *bf, hipStream_t s);
void bf2d_finish(fio_bf_s *bf, hipStream_t s);
void bf2d_apply(fio_bf_s *bf, bool adj, const double2 *X, long ldx, double2 *Y, long ldy, int nrhs, fio_prec prec,
                void *ws, bool freq_internal, hipStream_t s);
// permutation between user order and Morton order of a 2D grid (bf2d.hip)
void permute2d(int n, bool to_internal, const double2 *X, long ldx, double2 *Y, long ldy, int nrhs, hipStream_t s);
size_t bf_ws_bytes(const fio_bf_s *bf, int nrhs, fio_prec prec);
// column bucket of the tuned configurations: the next power of two of nrhs, capped at 64
int tile_key(bool adj, fio_prec prec, int nrhs);
// the tuned configuration for an apply (all zero when none was tuned)
TileCfg bf_tile(const fio_bf_s *bf, bool adj, fio_prec prec, int nrhs);
size_t bf_tw_off(const fio_bf_s *bf, bool cside, int lev);   // element offset of a level's twiddles
}  // namespace fio
