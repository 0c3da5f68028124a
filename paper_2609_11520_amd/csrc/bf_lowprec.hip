// Split-FP16 butterfly transfer passes on the matrix cores (gfx950 MFMA, FP32 accumulation).
//
// Growth direction of the solve (the low-precision K~^* of the refinement): every transfer
// block of eq. bf (a 2q x 2q complex block per group, Section 2.2) is applied as a real
// matrix product on v_mfma_f32_16x16x32_f16 with both operands split into a high and a low
// half-precision part, a = a_hi + a_lo, x = x_hi + x_lo, and
//     a x ~= a_hi x_hi + a_hi x_lo + a_lo x_hi      (the a_lo x_lo term is below FP32 rounding),
// all three products accumulated in FP32.  The middle factor is folded into the transfer
// level next to it (FP64 products before the split); the leaf factors stay in FP32 on the
// vector units.  Only q = 9 is built.
//
// Block storage (per transfer level, per direction, per group g; 32-bit words, each word a
// pair of halves (low half, high half)):
//     words [((g 2 + plane) 18 + row) 20 + col],  plane 0 = hi, 1 = lo,  col 18, 19 = 0,
// holding conj(e) = (Re e, -Im e) of the entry e = block(row, col).  Forward blocks have rows =
// forward output index c_out q + r, columns = input index c_in q + t (the explicit FP64 block);
// adjoint blocks are the conjugate transposes (rows = forward input index).
//
// MFMA mapping of one group (18 complex outputs, 18 complex inputs, 16 RHS columns per tile):
// real output row o = 2 i + part (part 0 = real, 1 = imaginary part of output i), 3 tiles of 16
// rows (36 used).  The K axis holds three regions (hi x hi, hi x lo, lo x hi) of 40 halves each
// (20 complex inputs as (re, im) pairs, 18 used), i.e. 15 slots of 8 halves over 4 K-tiles of
// 32; slot s = 4 kt + (lane / 16) of a lane is region s / 5 at input t0 = 4 (s mod 5).  Row
// 2i reads (Re a, -Im a) = the stored word; row 2i+1 reads (Im a, Re a), the stored word with
// its halves swapped and the new low half negated.  Both operands use the same slot map, so
// the sum over K is independent of how the instruction orders K inside a lane.
#include <type_traits>

#include "bf_apply.h"

namespace fio {

namespace {

constexpr int kQ = 9, kQ2 = 18, kCols = 20;
constexpr int kPlaneWords = kQ2 * kCols;          // 360
constexpr int kGroupWords = 2 * kPlaneWords;      // 720 words = 2880 bytes = 180 uint4

typedef _Float16 h8 __attribute__((ext_vector_type(8)));
typedef float f4 __attribute__((ext_vector_type(4)));
typedef unsigned u4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ uint32_t pack_h2(_Float16 lo, _Float16 hi) {
    return (uint32_t)__builtin_bit_cast(uint16_t, lo) | ((uint32_t)__builtin_bit_cast(uint16_t, hi) << 16);
}

typedef _Float16 h2 __attribute__((ext_vector_type(2)));

// x = hi + lo: hi truncated to half precision (so that x - hi is exact in FP32), lo rounded to
// nearest.  The remainder x - hi is one v_fma_mix_f32 per component (the half operand is widened
// inside the instruction; the exact result is representable, so the FMA does not round).
__device__ __forceinline__ void split2(float re, float im, uint32_t &hi, uint32_t &lo) {
    hi = __builtin_bit_cast(uint32_t, __builtin_amdgcn_cvt_pkrtz(re, im));
    float rr, ri;
    asm("v_fma_mix_f32 %0, %1, -1.0, %2 op_sel_hi:[1,0,0]" : "=v"(rr) : "v"(hi), "v"(re));
    asm("v_fma_mix_f32 %0, %1, -1.0, %2 op_sel:[1,0,0] op_sel_hi:[1,0,0]" : "=v"(ri) : "v"(hi), "v"(im));
    h2 l;
    l[0] = (_Float16)rr;
    l[1] = (_Float16)ri;
    lo = __builtin_bit_cast(uint32_t, l);
}

// ---------------------------------------------------------------------------
// block generation from the explicit FP64 transfer blocks (Section 2.2 entries).  With M64
// set, the middle factor is folded into the level next to it: the forward blocks of C^[h+1]
// become diag(M_p0, M_p1) A (p0, p1 the group's output pairs), the adjoint blocks of
// B^[h+1] become diag(M_p0^*, M_p1^*) A^* (p0, p1 the adjoint's output pairs), so that no
// pass applies M separately.  G is the number of groups per parent box of the level.
__global__ void gen_split(const double2 *__restrict__ A64, const double2 *__restrict__ M64, long G, long ngroups,
                          int adj, uint32_t *__restrict__ out) {
    const size_t id = blockIdx.x * (size_t)blockDim.x + threadIdx.x;
    if (id >= (size_t)ngroups * kPlaneWords) return;
    const int col = id % kCols, row = (id / kCols) % kQ2;
    const size_t g = id / kPlaneWords;
    const double2 *blk = A64 + g * kQ2 * kQ2;
    // entry e(row, col) of the applied block: forward A(row, col), adjoint conj(A(col, row))
    auto entry = [&](int r, int c) {
        const double2 v = adj ? blk[(size_t)c * kQ2 + r] : blk[(size_t)r * kQ2 + c];
        return adj ? zc(v.x, -v.y) : v;
    };
    double2 e = zc(0.0, 0.0);
    if (col < kQ2) {
        if (M64) {
            const int c = row / kQ, i = row % kQ;
            const long alpha = g / G, sigma = g % G;
            const long p = adj ? alpha * 2 * G + 2 * sigma + c : 2 * alpha * G + sigma + c * G;
            const double2 *m = M64 + (size_t)p * kQ * kQ;
            for (int j = 0; j < kQ; ++j) {
                // forward: M_p(i, j); adjoint: conj(M_p(j, i))
                const double2 mv = adj ? zc(m[j * kQ + i].x, -m[j * kQ + i].y) : m[i * kQ + j];
                const double2 a = entry(c * kQ + j, col);
                e.x += mv.x * a.x - mv.y * a.y;
                e.y += mv.x * a.y + mv.y * a.x;
            }
        } else {
            e = entry(row, col);
        }
    }
    // stored: conj(e)
    const double re = e.x, im = -e.y;
    const _Float16 hr = (_Float16)(float)re, hi_ = (_Float16)(float)im;
    const _Float16 lr = (_Float16)(float)(re - (double)hr), li = (_Float16)(float)(im - (double)hi_);
    uint32_t *o = out + g * kGroupWords + (size_t)row * kCols + col;
    o[0] = pack_h2(hr, hi_);
    o[kPlaneWords] = pack_h2(lr, li);
}

// ---------------------------------------------------------------------------
// Fused split pass: the sub-butterfly decomposition of the structured passes (KL factors on
// closed subproblems of 2^KL pairs, 64 right-hand sides per workgroup, lane = column while
// loading and storing).  Between factors the coefficients live in LDS as hi/lo half planes,
// pre-scaled per column by a power of two that puts the column's largest input entry in
// [16, 32): three factors can grow entries by at most ~(2 * 3)^3, well inside half range, and
// the smallest representable low part stays ~2^-29 below the column maximum.
//
// LDS pair slots are permuted so that at every factor group g reads slots 2g and 2g + 1 (in
// the forward direction the natural order already has this property; the adjoint writes each
// output pair to the slot where the next factor reads it): every B-operand address is then a
// per-lane constant.  The blocks of the next factor are fetched into registers during the
// current one and staged in LDS in two forms, as stored (even rows) and transformed for odd
// rows, so the operand transform is paid once per workgroup instead of once per wave.
// Wave 2 g + h computes group g for columns [32 h, 32 h + 32) (two 16-column tiles).  The last
// factor writes FP32 results in natural pair order (aliasing the planes), which are unscaled
// and stored.
struct SplitArgsK {
    const u4 *A[3];
    long G0;
    const float2 *in;
    float2 *out;
    int nrhs;
};

// slot of local pair p at forward step j of a pass of 2^KL pairs (see above)
template <int KL, bool ADJ> __device__ __forceinline__ int split_slot(int j, int p) {
    if (!ADJ) return p;
    const int Gl = (1 << KL) >> (j + 1);
    const int hi = p / Gl;
    return 2 * ((hi >> 1) * Gl + p % Gl) + (hi & 1);
}

// LDS planes: group g's two input pairs occupy 20 rows (slot 2g + c, coefficient i at row
// 20 g + 9 c + i; rows 18, 19 stay zero), each row holds 64 columns with bits 4-5 of the column
// index XORed with bits 2-3 of the row, so that the four quarter-waves of an operand read (rows
// 4 apart) and of an output write (rows 2 apart) mostly fall into different bank ranges
__device__ __forceinline__ int prow(int slot, int i) { return 20 * (slot >> 1) + kQ * (slot & 1) + i; }
__device__ __forceinline__ int pidx(int row, int n) { return row * 64 + (n ^ (((row >> 2) & 3) << 4)); }

__device__ __forceinline__ u4 odd_form(u4 w) {
    // odd rows read (Im a, Re a): swap the halves of the stored (Re a, -Im a), negate the low one
    w.x = __builtin_amdgcn_alignbit(w.x, w.x, 16) ^ 0x8000u;
    w.y = __builtin_amdgcn_alignbit(w.y, w.y, 16) ^ 0x8000u;
    w.z = __builtin_amdgcn_alignbit(w.z, w.z, 16) ^ 0x8000u;
    w.w = __builtin_amdgcn_alignbit(w.w, w.w, 16) ^ 0x8000u;
    return w;
}

template <int KL, bool ADJ>
__global__ void __launch_bounds__((1 << KL) * 64, 4) k_split_fused(SplitArgsK a) {
    using C = float2;
    constexpr int Q = kQ, P = 1 << KL, NG = P / 2, PW = NG * 20 * 64, NT = P * 64;
    constexpr int BLK4 = kGroupWords / 4;      // uint4 per group block
    constexpr int NSTG = (NG * BLK4 + NT - 1) / NT;
    constexpr int ZERO = 2 * PW;
    __shared__ uint32_t sm[2 * PW + 256];      // hi plane, lo plane (swizzled, see pidx), 256 zero words
    // [even / odd-row form][group][block]; the odd form starts 8 words (mod 64) after the even
    // one, so lanes 2r and 2r + 1, which read the same row in the two forms, use different banks
    constexpr int SAF = NG * BLK4 + 2;
    __shared__ u4 sA[2 * SAF];
    __shared__ float cmax[P][64];
    C *ftile = reinterpret_cast<C *>(sm);      // [P Q rows][64] FP32 results of the last factor (pidx)
    static_assert(P * Q * 64 * 2 <= 2 * PW, "the FP32 tile aliases the planes");
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int col = blockIdx.y * 64 + lane;
    const bool act = col < a.nrhs;
    const long nS = (2 * a.G0) >> KL;
    const long A = blockIdx.x / nS, S = blockIdx.x % nS;
    const long Glast = a.G0 >> (KL - 1);
    const size_t ld = (size_t)a.nrhs;

    // global index of entry e of the staged blocks of forward step j
    auto blk_src = [&](int j, int e) {
        const int b = e / BLK4, o = e % BLK4;
        const int Gl = P >> (j + 1);
        const long g = (A * (1L << j) + b / Gl) * (a.G0 >> j) + S * Gl + b % Gl;
        return a.A[j] + (size_t)g * BLK4 + o;
    };
    // Loads carry no branch (out-of-range threads read a valid element and discard it): a load
    // under a thread condition sits in a block of its own, and the wait for it comes before the
    // next load is issued.
    u4 pf[NSTG];
    {
        const int j0 = ADJ ? KL - 1 : 0;
#pragma unroll
        for (int r = 0; r < NSTG; ++r) {
            const int e = tid + r * NT;
            pf[r] = *blk_src(j0, e < NG * BLK4 ? e : 0);
        }
    }
    // load pair `wave`, scale per column, split into the planes at the first factor's slots
    float inv;
    {
        const int lp = wave;
        const long gp = ADJ ? (A * P + lp) * Glast + S : A * 2 * a.G0 + S * P + lp;
        const C *src = a.in + (size_t)gp * Q * ld + (act ? col : (int)blockIdx.y * 64);
        C v[Q];
        float m = 0.f;
#pragma unroll
        for (int i = 0; i < Q; ++i) v[i] = src[i * ld];
#pragma unroll
        for (int i = 0; i < Q; ++i) {
            if (!act) v[i] = make_float2(0.f, 0.f);
            m = fmaxf(m, fmaxf(fabsf(v[i].x), fabsf(v[i].y)));
        }
        cmax[lp][lane] = m;
        for (int e = tid; e < 256; e += NT) sm[ZERO + e] = 0u;
        // the two padding rows of every group, both planes
        for (int e = tid; e < NG * 2 * 64 * 2; e += NT) {
            const int pl = e / (NG * 128), r = (e / 64) % (NG * 2);
            sm[pl * PW + (20 * (r >> 1) + kQ2 + (r & 1)) * 64 + (e & 63)] = 0u;
        }
#pragma unroll
        for (int r = 0; r < NSTG; ++r) {
            const int e = tid + r * NT;
            if (e < NG * BLK4) {
                sA[e] = pf[r];
                sA[SAF + e] = odd_form(pf[r]);
            }
        }
        __syncthreads();
        float mm = 0.f;
#pragma unroll
        for (int w = 0; w < P; ++w) mm = fmaxf(mm, cmax[w][lane]);
        int e;
        (void)frexpf(mm, &e);
        e = e < -100 ? -100 : (e > 100 ? 100 : e);
        const float sc = ldexpf(1.f, 5 - e);
        inv = ldexpf(1.f, e - 5);
        const int slot = split_slot<KL, ADJ>(ADJ ? KL - 1 : 0, lp);
#pragma unroll
        for (int i = 0; i < Q; ++i) {
            uint32_t hi, lo;
            split2(v[i].x * sc, v[i].y * sc, hi, lo);
            sm[pidx(prow(slot, i), lane)] = hi;
            sm[PW + pidx(prow(slot, i), lane)] = lo;
        }
    }
    __syncthreads();

    const int grp = wave >> 1, nh = wave & 1;
    const int r16 = lane & 15, qd = lane >> 4;
    // per-lane constant operand offsets: B word of K-tile kt, input t0 of the first 16-column
    // tile (input t0 + e4 is 64 e4 further, since rows 20 g + t0 .. + 3 share their swizzle; the
    // second tile's word differs in column bit 4: offset ^ 16), A uint4s of (row tile mt, K-tile
    // kt) inside the group's staged block
    int boff[4], aoff[3][4];
#pragma unroll
    for (int kt = 0; kt < 4; ++kt) {
        const int sl = 4 * kt + qd, reg = sl / 5, t0 = 4 * (sl % 5);
        boff[kt] = reg == 3 ? ZERO + r16 : (reg == 1 ? PW : 0) + pidx(20 * grp + t0, nh * 32 + r16);
#pragma unroll
        for (int mt = 0; mt < 3; ++mt) {
            const int ir = (16 * mt + r16) >> 1, i = ir < kQ2 ? ir : kQ2 - 1;
            aoff[mt][kt] = ((reg == 2 ? 1 : 0) * kQ2 + i) * (kCols / 4) + (reg < 3 ? t0 / 4 : 0);
        }
    }
    const u4 *blkA = sA + (lane & 1) * SAF + grp * BLK4;
#pragma unroll
    for (int st = 0; st < KL; ++st) {
        const int j = ADJ ? KL - 1 - st : st;
        const int Gl = P >> (j + 1);
        const int aj = grp / Gl, sj = grp % Gl;
        const int lin0 = aj * 2 * Gl + 2 * sj, lout0 = 2 * aj * Gl + sj;
        const int d0 = ADJ ? lin0 : lout0, d1 = ADJ ? lin0 + 1 : lout0 + Gl;
        if (st + 1 < KL) {
            const int jn = ADJ ? j - 1 : j + 1;
#pragma unroll
            for (int r = 0; r < NSTG; ++r) {
                const int e = tid + r * NT;
                pf[r] = *blk_src(jn, e < NG * BLK4 ? e : 0);
            }
        }
        u4 Bop[2][4];
#pragma unroll
        for (int nt = 0; nt < 2; ++nt)
#pragma unroll
            for (int kt = 0; kt < 4; ++kt) {
                const uint32_t *bp = sm + (boff[kt] ^ (nt * 16));
                Bop[nt][kt] = u4{bp[0], bp[64], bp[128], bp[192]};
            }
        f4 acc[2][3];
#pragma unroll
        for (int mt = 0; mt < 3; ++mt) {
            u4 Aop[4];
#pragma unroll
            for (int kt = 0; kt < 4; ++kt) Aop[kt] = blkA[aoff[mt][kt]];
#pragma unroll
            for (int nt = 0; nt < 2; ++nt) {
                f4 c4 = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
                for (int kt = 0; kt < 4; ++kt)
                    c4 = __builtin_amdgcn_mfma_f32_16x16x32_f16(__builtin_bit_cast(h8, Aop[kt]),
                                                               __builtin_bit_cast(h8, Bop[nt][kt]), c4, 0, 0, 0);
                acc[nt][mt] = c4;
            }
        }
        __syncthreads();
        // outputs: lane holds rows 16 mt + 4 qd .. + 3 = (re, im) of outputs i0, i0 + 1 of its
        // column; they go to the next factor's slots (natural order after the last factor)
        const int e0 = st + 1 < KL ? split_slot<KL, ADJ>(ADJ ? j - 1 : j + 1, d0) : d0;
        const int e1 = st + 1 < KL ? split_slot<KL, ADJ>(ADJ ? j - 1 : j + 1, d1) : d1;
#pragma unroll
        for (int nt = 0; nt < 2; ++nt) {
            const int n = nh * 32 + nt * 16 + r16;
#pragma unroll
            for (int mt = 0; mt < 3; ++mt) {
#pragma unroll
                for (int u = 0; u < 2; ++u) {
                    const int i = 8 * mt + 2 * qd + u;
                    if (i < kQ2) {
                        const int c = i >= Q, jj = i - Q * c;
                        const int w = pidx(prow(c ? e1 : e0, jj), n);
                        const float re = u ? acc[nt][mt].z : acc[nt][mt].x;
                        const float im = u ? acc[nt][mt].w : acc[nt][mt].y;
                        if (st == KL - 1) {
                            ftile[pidx((c ? e1 : e0) * Q + jj, n)] = make_float2(re, im);
                        } else {
                            uint32_t hi, lo;
                            split2(re, im, hi, lo);
                            sm[w] = hi;
                            sm[PW + w] = lo;
                        }
                    }
                }
            }
        }
        if (st + 1 < KL) {
#pragma unroll
            for (int r = 0; r < NSTG; ++r) {
                const int e = tid + r * NT;
                if (e < NG * BLK4) {
                    sA[e] = pf[r];
                    sA[SAF + e] = odd_form(pf[r]);
                }
            }
            __syncthreads();
        }
    }
    {
        // The last factor of wave 2 g + h wrote output pairs 2 g and 2 g + 1 (both directions) for
        // columns [32 h, 32 h + 32); the wave stores exactly these (lanes 0-31 the first pair,
        // 32-63 the second), reading back only its own writes, so no barrier precedes the store.
        const int lp = 2 * grp + (lane >> 5), n = nh * 32 + (lane & 31);
        const float invn = __shfl(inv, n);
        const long gp = ADJ ? A * 2 * a.G0 + S * P + lp : (A * P + lp) * Glast + S;
        C *dstp = a.out + (size_t)gp * Q * ld + (size_t)blockIdx.y * 64 + n;
        const bool actn = (int)(blockIdx.y * 64 + n) < a.nrhs;
#pragma unroll
        for (int i = 0; i < Q; ++i)
            if (actn) dstp[i * ld] = cscale(ftile[pidx(lp * Q + i, n)], invn);
    }
}

template <int KL>
void launch_split(const SplitArgsK &k, bool adj, long N, hipStream_t s) {
    dim3 grid((unsigned)(N >> KL), (unsigned)((k.nrhs + 63) / 64));
    dim3 block((1 << KL) * 64);
    if (adj)
        k_split_fused<KL, true><<<grid, block, 0, s>>>(k);
    else
        k_split_fused<KL, false><<<grid, block, 0, s>>>(k);
}

size_t split_level_words(const fio_bf_s *bf) { return (size_t)(bf->N / 2) * kGroupWords; }

}  // namespace

// words offset of level `lev` (0 = level h+1) of side B (cside = false) or C, forward or adjoint copy
static size_t split_off(const fio_bf_s *bf, bool cside, int lev, bool adj) {
    return ((size_t)(lev * 2 + (cside ? 1 : 0)) * 2 + (adj ? 1 : 0)) * split_level_words(bf);
}

const void *split_blocks(const fio_bf_s *bf, bool cside, int lev, bool adj) {
    return bf->f16.as<uint32_t>() + split_off(bf, cside, lev, adj);
}

void split_pass(const SplitPass &sp, int kl, bool adj, long N, hipStream_t s) {
    SplitArgsK k;
    for (int j = 0; j < 3; ++j) k.A[j] = reinterpret_cast<const u4 *>(sp.A[j]);
    k.G0 = sp.G0;
    k.in = sp.in;
    k.out = sp.out;
    k.nrhs = sp.nrhs;
    switch (kl) {
        case 1: launch_split<1>(k, adj, N, s); break;
        case 2: launch_split<2>(k, adj, N, s); break;
        case 3: launch_split<3>(k, adj, N, s); break;
        default: throw Err{FIO_ERR_UNSUPPORTED};
    }
}

// Builds the split copies of every transfer level (both directions) from the FP64 factors.
void bf_make_lowprec(fio_bf_s *bf, hipStream_t s) {
    if (bf->dim != 1 || bf->q != kQ) throw Err{FIO_ERR_UNSUPPORTED};
    if (bf->nl > 0) {
        bf->f16.alloc(split_off(bf, false, bf->nl, false) * sizeof(uint32_t));
        const long ng = bf->N / 2;
        const double2 *F = bf->f64.as<double2>();
        for (int lev = 0; lev < bf->nl; ++lev)
            for (int cs = 0; cs < 2; ++cs)
                for (int ad = 0; ad < 2; ++ad) {
                    // M folds into forward C^[h+1] and adjoint B^[h+1] (the passes next to M)
                    const bool fold = lev == 0 && (cs ? !ad : ad);
                    const long G = cs ? (1L << (bf->h + lev)) : (1L << (bf->L - bf->h - lev - 1));
                    gen_split<<<grid1d((size_t)ng * kPlaneWords, 256), 256, 0, s>>>(
                        F + (cs ? bf->offC[lev] : bf->offB[lev]), fold ? F + bf->offM : nullptr, G, ng, ad,
                        bf->f16.as<uint32_t>() + split_off(bf, cs != 0, lev, ad != 0));
                }
        FIO_HIP(hipGetLastError());
    }
    bf->split16 = true;
}

size_t bf_ws_bytes_split16(const fio_bf_s *bf, int nrhs) { return 2 * bf_coef_elems(bf, nrhs) * sizeof(float2); }

void bf_apply_f32(fio_bf_s *bf, bool adj, const double2 *X, long ldx, double2 *Y, long ldy, int nrhs,
                  const float2 *F, void *ws, hipStream_t s, bool split);

void bf_apply_split16(fio_bf_s *bf, bool adj, const double2 *X, long ldx, double2 *Y, long ldy, int nrhs,
                      void *ws, hipStream_t s) {
    bf_apply_f32(bf, adj, X, ldx, Y, ldy, nrhs, bf->f32.as<float2>(), ws, s, true);
}

}  // namespace fio
