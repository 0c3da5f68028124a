// Apply kernels of the butterfly factorization (Section 2.2, eq. bf), shared by the
// per-precision translation units bf_apply_f64.hip and bf_apply_f32.hip.
#pragma once
#include <type_traits>

#include "bf.h"
#include "timing.h"

namespace fio {

constexpr int kLeafPts = 8;
bool fused_disabled();
bool leaf_fused_disabled();

// Split-FP16 transfer passes on the matrix cores (bf_lowprec.hip): KL <= 3 transfer factors of
// one side per launch, FP32 coefficient buffers in and out, as the structured passes; the
// middle factor is folded into the blocks of the level next to it.
struct SplitPass {
    const void *A[3];        // split blocks of forward step j (forward or adjoint copy)
    long G0;
    const float2 *in;
    float2 *out;
    int nrhs;
};
void split_pass(const SplitPass &sp, int kl, bool adj, long N, hipStream_t s);
const void *split_blocks(const fio_bf_s *bf, bool cside, int lev, bool adj);

// ---------------------------------------------------------------------------
// geometry passed to the kernels by value
struct Geo {
    long N;
    int L, h, Lp, q, b, nsl;
    double c0, c1;
};


inline Geo geo_of(const fio_bf_s *bf) {
    return Geo{bf->N, bf->L, bf->h, bf->Lp, bf->q, bf->b, bf->nsl, bf->desc.c0, bf->desc.c1};
}

// ---------------------------------------------------------------------------
// apply kernels.  One thread per (unit, column); a unit is a leaf box, a
// transfer group or a middle-level pair.  Template Q = q keeps the 2q input
// and output coefficients of a unit in registers.
template <typename T> __device__ __forceinline__ cpx<T> ld_in(const double2 *p) {
    double2 v = *p;
    return cmake<cpx<T>>((T)v.x, (T)v.y);
}

// V (forward): coef[(tau 2^L' + sigma) q + j] = sum_s V[sigma][tau][j][s] x[sigma b + s]
template <typename T, int Q>
__global__ void k_leaf_in_fwd(Geo g, const cpx<T> *__restrict__ V, const double2 *__restrict__ X, long ldx,
                              cpx<T> *__restrict__ out, int nrhs) {
    using C = cpx<T>;
    size_t id = blockIdx.x * (size_t)blockDim.x + threadIdx.x;
    size_t nunit = (size_t)(1L << g.Lp) * g.nsl;
    if (id >= nunit * nrhs) return;
    int col = id % nrhs;
    size_t unit = id / nrhs;
    int tau = unit % g.nsl;
    long sigma = unit / g.nsl;
    C x[kLeafPts];
    const double2 *xp = X + (size_t)col * ldx + sigma * kLeafPts;
#pragma unroll
    for (int s = 0; s < kLeafPts; ++s) x[s] = ld_in<T>(xp + s);
    const C *blk = V + (sigma * g.nsl + tau) * (size_t)Q * kLeafPts;
    size_t p = (size_t)tau * (1L << g.Lp) + sigma;
    C *op = out + p * Q * nrhs + col;
#pragma unroll
    for (int j = 0; j < Q; ++j) {
        C acc = czero<C>();
#pragma unroll
        for (int s = 0; s < kLeafPts; ++s) cfma(acc, blk[j * kLeafPts + s], x[s]);
        op[(size_t)j * nrhs] = acc;
    }
}

// U^* (adjoint): coef[(tau nsl + sigma) q + i] = sum_s conj(U[tau][sigma][s][i]) u[tau b + s]
template <typename T, int Q>
__global__ void k_leaf_in_adj(Geo g, const cpx<T> *__restrict__ U, const double2 *__restrict__ X, long ldx,
                              cpx<T> *__restrict__ out, int nrhs) {
    using C = cpx<T>;
    size_t id = blockIdx.x * (size_t)blockDim.x + threadIdx.x;
    size_t nunit = (size_t)(1L << g.Lp) * g.nsl;
    if (id >= nunit * nrhs) return;
    int col = id % nrhs;
    size_t unit = id / nrhs;              // = tau * nsl + sigma = pair index at U-level L'
    long tau = unit / g.nsl;
    C x[kLeafPts];
    const double2 *xp = X + (size_t)col * ldx + tau * kLeafPts;
#pragma unroll
    for (int s = 0; s < kLeafPts; ++s) x[s] = ld_in<T>(xp + s);
    const C *blk = U + unit * (size_t)kLeafPts * Q;
    C *op = out + unit * Q * nrhs + col;
#pragma unroll
    for (int i = 0; i < Q; ++i) {
        C acc = czero<C>();
#pragma unroll
        for (int s = 0; s < kLeafPts; ++s) cfmac(acc, blk[s * Q + i], x[s]);
        op[(size_t)i * nrhs] = acc;
    }
}

// One transfer factor (B or C, forward or conjugate-transposed).
// Group grp = alpha G + sigma; forward inputs at pairs alpha 2G + 2 sigma + c,
// outputs at pairs (2 alpha + c) G + sigma.
template <typename T, int Q, bool ADJ, bool UNI>
__global__ void __launch_bounds__(256) k_transfer(const cpx<T> *__restrict__ A, long G,
                                                  const cpx<T> *__restrict__ in, cpx<T> *__restrict__ out,
                                                  long ngroups, int nrhs) {
    using C = cpx<T>;
    constexpr int Q2 = 2 * Q;
    size_t id = blockIdx.x * (size_t)blockDim.x + threadIdx.x;
    if (id >= (size_t)ngroups * nrhs) return;
    int col = id % nrhs;
    long grp = id / nrhs;
    if (UNI) grp = __builtin_amdgcn_readfirstlane(grp);
    long alpha = grp / G, sigma = grp % G;
    size_t pin0 = alpha * 2 * G + 2 * sigma;          // pairs pin0, pin0 + 1
    size_t pout0 = 2 * alpha * G + sigma;             // pairs pout0, pout0 + G
    size_t src0 = ADJ ? pout0 : pin0, src1 = ADJ ? pout0 + G : pin0 + 1;
    size_t dst0 = ADJ ? pin0 : pout0, dst1 = ADJ ? pin0 + 1 : pout0 + G;
    C x[Q2];
#pragma unroll
    for (int t = 0; t < Q; ++t) {
        x[t] = in[(src0 * Q + t) * nrhs + col];
        x[Q + t] = in[(src1 * Q + t) * nrhs + col];
    }
    const C *a = A + (size_t)grp * Q2 * Q2;
#pragma unroll
    for (int r = 0; r < Q2; ++r) {
        C acc = czero<C>();
#pragma unroll
        for (int c = 0; c < Q2; ++c) {
            if (ADJ)
                cfmac(acc, a[c * Q2 + r], x[c]);
            else
                cfma(acc, a[r * Q2 + c], x[c]);
        }
        size_t dst = (r < Q) ? dst0 : dst1;
        out[(dst * Q + (r % Q)) * nrhs + col] = acc;
    }
}

template <typename T, int Q, bool ADJ, bool UNI>
__global__ void __launch_bounds__(256) k_middle(const cpx<T> *__restrict__ M, const cpx<T> *__restrict__ in,
                                                cpx<T> *__restrict__ out, long npairs, int nrhs) {
    using C = cpx<T>;
    size_t id = blockIdx.x * (size_t)blockDim.x + threadIdx.x;
    if (id >= (size_t)npairs * nrhs) return;
    int col = id % nrhs;
    long p = id / nrhs;
    if (UNI) p = __builtin_amdgcn_readfirstlane(p);
    C x[Q];
#pragma unroll
    for (int j = 0; j < Q; ++j) x[j] = in[(p * Q + j) * nrhs + col];
    const C *m = M + (size_t)p * Q * Q;
#pragma unroll
    for (int i = 0; i < Q; ++i) {
        C acc = czero<C>();
#pragma unroll
        for (int j = 0; j < Q; ++j) {
            if (ADJ)
                cfmac(acc, m[j * Q + i], x[j]);
            else
                cfma(acc, m[i * Q + j], x[j]);
        }
        out[(p * Q + i) * nrhs + col] = acc;
    }
}

// U (forward): y[tau b + s] = sum_sigma sum_i U[tau][sigma][s][i] coef[(tau nsl + sigma) q + i]
template <typename T, int Q>
__global__ void k_leaf_out_fwd(Geo g, const cpx<T> *__restrict__ U, const cpx<T> *__restrict__ in,
                               double2 *__restrict__ Y, long ldy, int nrhs, const double2 *__restrict__ Ysub,
                               long ldsub) {
    using C = cpx<T>;
    size_t id = blockIdx.x * (size_t)blockDim.x + threadIdx.x;
    size_t nunit = (size_t)1 << g.Lp;
    if (id >= nunit * nrhs) return;
    int col = id % nrhs;
    long tau = id / nrhs;
    C acc[kLeafPts];
#pragma unroll
    for (int s = 0; s < kLeafPts; ++s) acc[s] = czero<C>();
    for (int sg = 0; sg < g.nsl; ++sg) {
        size_t p = (size_t)tau * g.nsl + sg;
        C d[Q];
#pragma unroll
        for (int i = 0; i < Q; ++i) d[i] = in[(p * Q + i) * nrhs + col];
        const C *blk = U + p * (size_t)kLeafPts * Q;
#pragma unroll
        for (int s = 0; s < kLeafPts; ++s) {
#pragma unroll
            for (int i = 0; i < Q; ++i) cfma(acc[s], blk[s * Q + i], d[i]);
        }
    }
    double2 *yp = Y + (size_t)col * ldy + tau * kLeafPts;
    if (Ysub) {
        // Y = Ysub - (the apply), the residual of a refinement step
        const double2 *up = Ysub + (size_t)col * ldsub + tau * kLeafPts;
#pragma unroll
        for (int s = 0; s < kLeafPts; ++s) {
            const double2 u = up[s];
            yp[s] = zc(u.x - (double)acc[s].x, u.y - (double)acc[s].y);
        }
        return;
    }
#pragma unroll
    for (int s = 0; s < kLeafPts; ++s) yp[s] = zc((double)acc[s].x, (double)acc[s].y);
}

// V^* (adjoint): f[sigma b + s] = sum_tau sum_j conj(V[sigma][tau][j][s]) coef[(tau 2^L' + sigma) q + j]
template <typename T, int Q>
__global__ void k_leaf_out_adj(Geo g, const cpx<T> *__restrict__ V, const cpx<T> *__restrict__ in,
                               double2 *__restrict__ Y, long ldy, int nrhs) {
    using C = cpx<T>;
    size_t id = blockIdx.x * (size_t)blockDim.x + threadIdx.x;
    size_t nunit = (size_t)1 << g.Lp;
    if (id >= nunit * nrhs) return;
    int col = id % nrhs;
    long sigma = id / nrhs;
    C acc[kLeafPts];
#pragma unroll
    for (int s = 0; s < kLeafPts; ++s) acc[s] = czero<C>();
    for (int t = 0; t < g.nsl; ++t) {
        size_t p = (size_t)t * (1L << g.Lp) + sigma;
        C c[Q];
#pragma unroll
        for (int j = 0; j < Q; ++j) c[j] = in[(p * Q + j) * nrhs + col];
        const C *blk = V + ((size_t)sigma * g.nsl + t) * Q * kLeafPts;
#pragma unroll
        for (int j = 0; j < Q; ++j)
#pragma unroll
            for (int s = 0; s < kLeafPts; ++s) cfmac(acc[s], blk[j * kLeafPts + s], c[j]);
    }
    double2 *yp = Y + (size_t)col * ldy + sigma * kLeafPts;
#pragma unroll
    for (int s = 0; s < kLeafPts; ++s) yp[s] = zc((double)acc[s].x, (double)acc[s].y);
}

// ---------------------------------------------------------------------------
// Fused transfer pass: KL consecutive transfer factors on closed sub-butterflies.
// In the pair numbering of the first factor of a pass (G0 = number of sigma per
// alpha there), subproblem (A, S) owns the 2^KL input pairs A 2 G0 + S 2^KL + b
// and, after KL factors, the 2^KL output pairs (A 2^KL + a) (G0 / 2^(KL-1)) + S;
// every intermediate pair stays inside the subproblem.  A workgroup of 2^KL
// waves keeps the subproblem's coefficients for 64 right-hand sides in LDS
// (lane = column); at every factor two waves share one 2q x 2q block (q output
// rows each), read through the scalar cache (the block index is uniform per
// wave) after the whole workgroup has pulled the step's blocks into L2.  ADJ runs the
// pass backwards with conjugate-transposed blocks.  EPI_M applies the middle
// factor (or its adjoint) to the pass's output pairs before they are stored.
template <typename T> struct FusedArgs {
    const cpx<T> *A[4];      // factor array of forward step j
    const cpx<T> *M;         // middle factor (EPI_M)
    long G0;
    const cpx<T> *in;
    cpx<T> *out;
    int nrhs;
    int sink;                // always 0 (keeps the L2 warm-up loads alive)
    double *sink_ptr;
};

template <typename T, int Q, int KL, bool ADJ, bool EPI_M>
__global__ void __launch_bounds__((1 << KL) * 64, 4) k_transfer_fused(FusedArgs<T> a) {
    using C = cpx<T>;
    constexpr int P = 1 << KL, NG = P / 2, NW = P, Q2 = 2 * Q;
    __shared__ C lds[P * Q * 64];
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int col = blockIdx.y * 64 + lane;
    const bool act = col < a.nrhs;
    const long nS = (2 * a.G0) >> KL;
    const long A = blockIdx.x / nS, S = blockIdx.x % nS;
    const long Glast = a.G0 >> (KL - 1);
    const size_t ld = (size_t)a.nrhs;
    // L2 prefetch of a step's factor blocks: every thread loads a few 16-byte chunks of the
    // step's NG blocks into registers; they are consumed (stored only when sink != 0, i.e.
    // never) after the step's compute, so the loads overlap it and the scalar loads of the
    // following step hit L2.
    constexpr int NT = 64 * P;
    constexpr int CPB = (int)((size_t)Q2 * Q2 * sizeof(C) / 16);   // 16-byte chunks per block
    constexpr int NPF = (NG * CPB + NT - 1) / NT;
    double2 pf[NPF];
    auto issue = [&](int j) {
        const int Gl = P >> (j + 1);
        const long Gj = a.G0 >> j;
#pragma unroll
        for (int k = 0; k < NPF; ++k) {
            const int e = tid + k * NT;
            pf[k] = zc(0.0, 0.0);
            if (e < NG * CPB) {
                const int b = e / CPB, off = e % CPB;
                const long g = (A * (1L << j) + b / Gl) * Gj + S * Gl + b % Gl;
                pf[k] = reinterpret_cast<const double2 *>(a.A[j] + (size_t)g * Q2 * Q2)[off];
            }
        }
    };
    auto consume = [&]() {
        if (a.sink) {
#pragma unroll
            for (int k = 0; k < NPF; ++k) a.sink_ptr[tid * NPF + k] = pf[k].x + pf[k].y;
        }
    };
    issue(ADJ ? KL - 1 : 0);
    // load: forward input positions (or forward output positions for ADJ)
    for (int lp = wave; lp < P; lp += NW) {
        const long gp = ADJ ? (A * P + lp) * Glast + S : A * 2 * a.G0 + S * P + lp;
        const C *src = a.in + (size_t)gp * Q * ld + col;
#pragma unroll
        for (int i = 0; i < Q; ++i) lds[(lp * Q + i) * 64 + lane] = act ? src[i * ld] : czero<C>();
    }
    __syncthreads();
    // two waves per group: wave = 2 * group + half, half selects output rows [half Q, half Q + Q)
    const int grp = wave >> 1, half = wave & 1;
#pragma unroll
    for (int st = 0; st < KL; ++st) {
        const int j = ADJ ? KL - 1 - st : st;
        consume();
        if (st + 1 < KL) issue(ADJ ? j - 1 : j + 1);
        const int Gl = P >> (j + 1);
        const long Gj = a.G0 >> j;
        const int aj = grp / Gl, sj = grp % Gl;
        const long g = (A * (1L << j) + aj) * Gj + (S * Gl + sj);
        const int lin0 = aj * 2 * Gl + 2 * sj, lout0 = 2 * aj * Gl + sj;
        const int src0 = ADJ ? lout0 : lin0, src1 = ADJ ? lout0 + Gl : lin0 + 1;
        const int dst = half ? (ADJ ? lin0 + 1 : lout0 + Gl) : (ADJ ? lin0 : lout0);
        C x[Q2];
#pragma unroll
        for (int t = 0; t < Q; ++t) {
            x[t] = lds[(src0 * Q + t) * 64 + lane];
            x[Q + t] = lds[(src1 * Q + t) * 64 + lane];
        }
        __syncthreads();
        const C *blk = a.A[j] + (size_t)g * Q2 * Q2;
#pragma unroll 1
        for (int rr = 0; rr < Q; ++rr) {
            const int r = half * Q + rr;
            C acc = czero<C>();
#pragma unroll
            for (int c = 0; c < Q2; ++c) {
                if (ADJ)
                    cfmac(acc, blk[c * Q2 + r], x[c]);
                else
                    cfma(acc, blk[r * Q2 + c], x[c]);
            }
            lds[(dst * Q + rr) * 64 + lane] = acc;
        }
        __syncthreads();
    }
    // store: forward output positions (or forward input positions for ADJ); one pair per wave
    for (int lp = wave; lp < P; lp += NW) {
        const long gp = ADJ ? A * 2 * a.G0 + S * P + lp : (A * P + lp) * Glast + S;
        C *dstp = a.out + (size_t)gp * Q * ld + col;
        if (EPI_M) {
            C x[Q];
#pragma unroll
            for (int i = 0; i < Q; ++i) x[i] = lds[(lp * Q + i) * 64 + lane];
            const C *m = a.M + (size_t)gp * Q * Q;
#pragma unroll
            for (int i = 0; i < Q; ++i) {
                C acc = czero<C>();
#pragma unroll
                for (int jj = 0; jj < Q; ++jj) {
                    if (ADJ)
                        cfmac(acc, m[jj * Q + i], x[jj]);
                    else
                        cfma(acc, m[i * Q + jj], x[jj]);
                }
                if (act) dstp[i * ld] = acc;
            }
        } else {
#pragma unroll
            for (int i = 0; i < Q; ++i)
                if (act) dstp[i * ld] = lds[(lp * Q + i) * 64 + lane];
        }
    }
}

template <typename T, int Q, int KL>
static void launch_fused(const FusedArgs<T> &fa, bool adj, bool epi, long N, hipStream_t s) {
    dim3 grid((unsigned)(N >> KL), (unsigned)((fa.nrhs + 63) / 64));
    dim3 block((1 << KL) * 64);
    if (adj) {
        if (epi)
            k_transfer_fused<T, Q, KL, true, true><<<grid, block, 0, s>>>(fa);
        else
            k_transfer_fused<T, Q, KL, true, false><<<grid, block, 0, s>>>(fa);
    } else {
        if (epi)
            k_transfer_fused<T, Q, KL, false, true><<<grid, block, 0, s>>>(fa);
        else
            k_transfer_fused<T, Q, KL, false, false><<<grid, block, 0, s>>>(fa);
    }
}

// largest pass length whose LDS tile fits (two workgroups per CU)
template <typename T, int Q> constexpr int fused_max_kl() {
    return ((size_t)8 * Q * 64 * sizeof(cpx<T>) <= 80 * 1024) ? 3 : 2;
}

template <typename T, int Q>
static void run_fused(const FusedArgs<T> &fa, int kl, bool adj, bool epi, long N, hipStream_t s) {
    switch (kl) {
        case 1: launch_fused<T, Q, 1>(fa, adj, epi, N, s); break;
        case 2: launch_fused<T, Q, 2>(fa, adj, epi, N, s); break;
        case 3:
            if constexpr (fused_max_kl<T, Q>() >= 3) {
                launch_fused<T, Q, 3>(fa, adj, epi, N, s);
                break;
            }
            [[fallthrough]];
        default: throw Err{FIO_ERR_UNSUPPORTED};
    }
}

template <int Q> constexpr bool fused_q() { return Q == 5 || Q == 9 || Q == 13; }

// Structured fused pass: same sub-butterfly decomposition as k_transfer_fused, with every
// 2q x 2q block applied as four quadrants diag(a) P diag(b) (see gen_TW_B / gen_TW_C):
// the per-group twiddles (8q complex) come through the scalar cache, the two shared q x q
// Lagrange matrices travel in the kernel arguments.  Wave 2g + h handles group g:
// forward it produces output child c_out = h, adjoint it produces input child c_in = h.
template <typename T, int Q> struct StructArgs {
    const cpx<T> *TW[4];     // twiddles of forward step j
    const cpx<T> *M;         // middle factor (EPI_M)
    long G0;
    const cpx<T> *in;
    cpx<T> *out;
    int nrhs;
    int cside;               // 1: C factors (P transposed, child index c_in)
    const cpx<T> *V;         // LEAF: the leaf factor, V^[L'] forward (blocks V[sigma][tau], q x 8),
                             // U^[L'] adjoint (blocks U[tau][sigma], 8 x q)
    const double2 *X;        // LEAF: the input block (column-major, leading dimension ldx)
    long ldx;
    T P[2][Q][Q];            // P_c(i, t)
    T PT[2][Q][Q];           // P_c(t, i): the transposes, so that every variant reads one pattern
    T SD[Q][Q];              // column t: S(r, t), r < (q+1)/2, then D(r, t), r < q/2 (see struct_step)
};

// One transfer factor of a structured pass for the calling wave: group grp of forward step j,
// output child h (forward) or input child h (adjoint), for the lane's column, from the tile in
// LDS (pair p, coefficient i at row p q + i, 64 columns per row) and the group's 8q twiddles
// at tw.  The result goes to acc; returns the local pair it belongs to.
template <typename T, int Q, int KL, bool ADJ, bool CS>
__device__ __forceinline__ int struct_step(const StructArgs<T, Q> &a, const cpx<T> *lds, const cpx<T> *tw, int grp,
                                           int h, int j, int lane, cpx<T> (&acc)[Q]) {
    using C = cpx<T>;
    constexpr int P = 1 << KL;
    // quadrant matrix M(r, t) = P_pc(r, t) (B side) or P_pc(t, r) (C side); the adjoint uses
    // M^T, so the stored matrix is read transposed when ADJ != CS
    constexpr bool TRANS = ADJ != CS;
    const int Gl = P >> (j + 1);
    const int aj = grp / Gl, sj = grp % Gl;
    const int lin0 = aj * 2 * Gl + 2 * sj, lout0 = 2 * aj * Gl + sj;
    // The output-side twiddle does not depend on the child summed over when the forward pass
    // runs C factors (a depends on c_out only) or the adjoint runs B factors (b depends on
    // c_in only): the two quadrant products are then summed first and scaled once.
    constexpr bool FACT = ADJ != CS;
#pragma unroll
    for (int r = 0; r < Q; ++r) acc[r] = czero<C>();
    // Element (r, t) of the quadrant matrix is read as Pm[t * Q + r], from P or its transpose as
    // the variant needs, one column t at a time: the products run with the input index outermost
    // (v_r += M(r, t) w_t for every r), so one scaled input and one column of the matrix are
    // live at a time; each v_r sums its terms in the order t = 0 .. Q-1.
    constexpr bool D = sizeof(T) == 8;
    if constexpr (!FACT) {
        // forward B side / adjoint C side: both quadrants use the same matrix (P_{c_out},
        // resp. P_{c_in}, c = h), so one pass over its columns serves both children
        const int s0 = ADJ ? lout0 : lin0, s1 = ADJ ? lout0 + Gl : lin0 + 1;
        const C *t0 = tw + (ADJ ? h * Q : h * 4 * Q);                  // quadrant o = 0
        const C *t1 = tw + (ADJ ? 4 * Q + h * Q : h * 4 * Q + Q);      // quadrant o = 1
        // a(c_out, c_in, .) at t_o, b(c_out, c_in, .) at t_o + 2 Q
        const T *Pm = (!TRANS ? &a.PT[0][0][0] : &a.P[0][0][0]) + h * Q * Q;
        C v0[Q], v1[Q];
#pragma unroll
        for (int r = 0; r < Q; ++r) v0[r] = v1[r] = czero<C>();
#pragma unroll
        for (int t = 0; t < Q; ++t) {
            // in double precision the column offset is opaque, so that each column's scalar
            // loads are issued with the column (the whole matrix at once would not fit the
            // scalar registers and would be spilled into vector lanes)
            int ot = t * Q;
            asm volatile("" : "+s"(ot));
            const C x0 = lds[(s0 * Q + t) * 64 + lane], x1 = lds[(s1 * Q + t) * 64 + lane];
            const C w0 = ADJ ? cmul(cconj(t0[t]), x0) : cmul(t0[2 * Q + t], x0);
            const C w1 = ADJ ? cmul(cconj(t1[t]), x1) : cmul(t1[2 * Q + t], x1);
#pragma unroll
            for (int r = 0; r < Q; ++r) {
                const T m = Pm[ot + r];
                v0[r].x = fma(m, w0.x, v0[r].x);
                v0[r].y = fma(m, w0.y, v0[r].y);
                v1[r].x = fma(m, w1.x, v1[r].x);
                v1[r].y = fma(m, w1.y, v1[r].y);
            }
        }
#pragma unroll
        for (int r = 0; r < Q; ++r) {
            if (ADJ) {
                cfmac(acc[r], t0[2 * Q + r], v0[r]);
                cfmac(acc[r], t1[2 * Q + r], v1[r]);
            } else {
                cfma(acc[r], t0[r], v0[r]);
                cfma(acc[r], t1[r], v1[r]);
            }
        }
    } else {
        // Both quadrants sum into one output through G_o = P_o^T, o = the child summed over
        // (forward: c_in, adjoint: c_out).  The Chebyshev points are symmetric about the box
        // centre, so P_1(i, t) = P_0(q-1-i, q-1-t), i.e. G_1 = J G_0 J with J the index reversal.
        // With z_t = w_1[q-1-t], s = w_0 + z and d = w_0 - z, rows r and r' = q-1-r of the sum
        // are S_r.s + D_r.d and S_r.s - D_r.d with S = (G_0(r, .) + G_0(r', .)) / 2 and
        // D = (G_0(r, .) - G_0(r', .)) / 2, and the middle row of odd q is G_0(m, .).s: half the
        // multiply-adds of the two separate quadrant products (StructArgs::SD holds S and D).
        constexpr int NS = (Q + 1) / 2, ND = Q / 2;
        const int c0out = ADJ ? 0 : h, c0in = ADJ ? h : 0, c1out = ADJ ? 1 : h, c1in = ADJ ? h : 1;
        const int src0 = ADJ ? lout0 : lin0, src1 = ADJ ? lout0 + Gl : lin0 + 1;
        // input-side twiddles: forward b(c_out, c_in, .), adjoint conj(a(c_out, c_in, .))
        const C *tw0 = tw + c0out * 4 * Q + (ADJ ? c0in : 2 + c0in) * Q;
        const C *tw1 = tw + c1out * 4 * Q + (ADJ ? c1in : 2 + c1in) * Q;
        C e[NS], f[ND];
#pragma unroll
        for (int r = 0; r < NS; ++r) e[r] = czero<C>();
#pragma unroll
        for (int r = 0; r < ND; ++r) f[r] = czero<C>();
#pragma unroll
        for (int t = 0; t < Q; ++t) {
            // one column of S and D per input index, loaded with the column (an opaque offset,
            // so that the whole matrix is not held in scalar registers)
            int ot = t * Q;
            asm volatile("" : "+s"(ot));
            const C x0 = lds[(src0 * Q + t) * 64 + lane], x1 = lds[(src1 * Q + (Q - 1 - t)) * 64 + lane];
            const C w0 = ADJ ? cmul(cconj(tw0[t]), x0) : cmul(tw0[t], x0);
            const C z = ADJ ? cmul(cconj(tw1[Q - 1 - t]), x1) : cmul(tw1[Q - 1 - t], x1);
            const C sv = cadd(w0, z), dv = csub(w0, z);
#pragma unroll
            for (int r = 0; r < NS; ++r) {
                const T m = (&a.SD[0][0])[ot + r];
                e[r].x = fma(m, sv.x, e[r].x);
                e[r].y = fma(m, sv.y, e[r].y);
            }
#pragma unroll
            for (int r = 0; r < ND; ++r) {
                const T m = (&a.SD[0][0])[ot + NS + r];
                f[r].x = fma(m, dv.x, f[r].x);
                f[r].y = fma(m, dv.y, f[r].y);
            }
        }
#pragma unroll
        for (int r = 0; r < ND; ++r) {
            acc[r] = cadd(e[r], f[r]);
            acc[Q - 1 - r] = csub(e[r], f[r]);
        }
        if constexpr (Q % 2 == 1) acc[ND] = e[ND];
    }
    if (FACT) {
        // forward C side: a(c_out, .) of either input child; adjoint B side: b(., c_in) of
        // either output child (the two stored copies are equal)
        const C *ts = ADJ ? tw + (2 + h) * Q : tw + h * 4 * Q;
#pragma unroll
        for (int r = 0; r < Q; ++r) acc[r] = ADJ ? cmul(cconj(ts[r]), acc[r]) : cmul(ts[r], acc[r]);
    }
    return ADJ ? lin0 + h : (h ? lout0 + Gl : lout0);
}

// Register budget: single precision keeps 8 waves per SIMD (four 37 KB workgroups per CU at
// KL = 3, <= 64 VGPRs), double precision 4 (two 74 KB workgroups, LDS-bound anyway).
// LEAF (first pass of 3 levels: forward C side or adjoint B side): the pass also applies the
// leaf factor (V^[L'] forward, U^[L']* adjoint), reading the input vectors instead of the leaf
// coefficients (see the load phase).
template <typename T, int Q, int KL, bool ADJ, bool EPI_M, bool CS, bool LEAF = false>
__global__ void __launch_bounds__((1 << KL) * 64, sizeof(T) == 4 ? 6 : 4) k_struct_fused(StructArgs<T, Q> a) {
    using C = cpx<T>;
    constexpr int P = 1 << KL, NG = P / 2;
    static_assert(!LEAF || (KL == 3 && CS != ADJ), "the leaf factor folds into a first 3-level pass");
    // double precision: the twiddles of the current factor's NG groups, fetched into registers
    // during the previous factor (vector loads) and read back from LDS as broadcasts; single
    // precision reads them through the scalar cache (its register budget has no room)
    constexpr bool TWL = true;
    constexpr int NTW = TWL ? NG * 8 * Q : 1;
    __shared__ C lds[P * Q * 64];
    __shared__ C stw[NTW];
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int col = blockIdx.y * 64 + lane;
    const bool act = col < a.nrhs;
    const long nS = (2 * a.G0) >> KL;
    long A, S;
    if constexpr (LEAF) {
        // the 8 workgroups that read the same 64 input rows (one per coarse partner: A forward,
        // S adjoint) are dispatched one after another on one XCD (workgroups go round-robin over
        // the 8 XCDs), so the rows come from HBM once and from that XCD's L2 after; needs
        // nS % 8 == 0 forward, nS == 8 and 8 | (number of A) adjoint
        const long b = blockIdx.x, k = b >> 3;
        if constexpr (!ADJ) {
            A = k & 7;
            S = ((k >> 3) << 3) | (b & 7);
        } else {
            S = k & 7;
            A = ((k >> 3) << 3) | (b & 7);
        }
    } else {
        A = blockIdx.x / nS;
        S = blockIdx.x % nS;
    }
    const long Glast = a.G0 >> (KL - 1);
    const size_t ld = (size_t)a.nrhs;
    static_assert(NTW <= P * 64, "one twiddle per thread");
    // twiddle e (local group e / 8q, entry e % 8q) of forward step j
    auto tw_src = [&](int j, int e) {
        const int b = e / (8 * Q), o = e % (8 * Q);
        const int Gl = P >> (j + 1);
        const long g = (A * (1L << j) + b / Gl) * (a.G0 >> j) + S * Gl + b % Gl;
        return a.TW[j][(size_t)g * 8 * Q + o];
    };
    C twn = czero<C>();
    constexpr int NMP = (Q * Q + 63) / 64;
    C mpf[NMP];
    // Loads carry no branch (out-of-range lanes read a valid element and discard it): a load
    // under a lane condition sits in a block of its own, and the wait for it comes before the
    // next load is issued, which serializes the round trips of the load phase.
    const C tw0 = tw_src(ADJ ? KL - 1 : 0, tid < NTW ? tid : 0);
    // When the pass applies M, the middle block of this wave's output pair is fetched into
    // registers for the store phase: in double precision before the load phase, so that its
    // latency overlaps the coefficients' (measured faster); in single precision during the last
    // factor (the registers held through the pass cost more there than the latency).
    auto fetch_m = [&]() {
        const long gpo = ADJ ? A * 2 * a.G0 + S * P + wave : (A * P + wave) * Glast + S;
        const C *msrc = a.M + (size_t)gpo * Q * Q;
#pragma unroll
        for (int k2 = 0; k2 < NMP; ++k2) mpf[k2] = msrc[lane + 64 * k2 < Q * Q ? lane + 64 * k2 : Q * Q - 1];
    };
    constexpr bool EARLY_M = EPI_M && sizeof(T) == 8;
    if constexpr (EARLY_M) fetch_m();
    if constexpr (LEAF) {
        // Forward, the input pairs are (coarse partner A, leaf boxes 8S .. 8S + 7): pair
        // A 2^L' + box holds V[box][A] applied to rows 8 box .. 8 box + 7 of the input.  Adjoint,
        // they are (leaf boxes 8A .. 8A + 7, coarse partner S): pair 8 box + S holds U[box][S]^*
        // applied to the same rows.  The workgroup stages its 64 rows of its 64 columns in the
        // tile (lanes along rows, coalesced), each wave takes its box's 8 rows for its lane's
        // column, and after a barrier writes the pair's q coefficients where the load would have
        // put them.  Same operations, in the same order, as the leaf kernel followed by the load.
        constexpr int XP = 65;                                   // padded column stride of the staged rows
        static_assert(64 * XP <= P * Q * 64, "the staged rows fit the tile");
        constexpr int VB = Q * kLeafPts, NVB = (VB + 63) / 64;   // entries of one leaf block, per lane
        const int cb = blockIdx.y * 64;
        const int ncol = a.nrhs - cb < 64 ? a.nrhs - cb : 64;
        const long box0 = ADJ ? A * P : S * P;                   // first leaf box of the workgroup
        const long box = box0 + wave;
        const long partner = ADJ ? S : A;
        // the wave's leaf block (nsl = 8 partners), fetched with vector loads while the rows are
        // staged, so that its latency overlaps theirs
        const C *blk = a.V + ((size_t)box * kLeafPts + partner) * VB;
        C vpf[NVB];
#pragma unroll
        for (int k2 = 0; k2 < NVB; ++k2) vpf[k2] = blk[lane + 64 * k2 < VB ? lane + 64 * k2 : VB - 1];
        const double2 *xs = a.X + (size_t)box0 * kLeafPts;
        constexpr int NXS = 64 * 64 / (P * 64);                  // staged elements per thread
        double2 xv[NXS];
#pragma unroll
        for (int q = 0; q < NXS; ++q) {
            const int e = tid + q * P * 64, r = e & 63, cc = e >> 6;
            xv[q] = xs[r + (size_t)(cb + (cc < ncol ? cc : 0)) * a.ldx];
        }
        if (TWL && tid < NTW) stw[tid] = tw0;
#pragma unroll
        for (int q = 0; q < NXS; ++q) {
            const int e = tid + q * P * 64, r = e & 63, cc = e >> 6;
            lds[cc * XP + r] = cc < ncol ? cmake<C>((T)xv[q].x, (T)xv[q].y) : czero<C>();
        }
        __syncthreads();
        C x[kLeafPts];
#pragma unroll
        for (int t = 0; t < kLeafPts; ++t) x[t] = lds[lane * XP + wave * kLeafPts + t];
        __syncthreads();
        // The staged rows are consumed: the block goes to the wave's own pair rows and is read
        // back as broadcasts; the q outputs stay in registers until every read is done, then
        // overwrite those rows (LDS runs one wave's accesses in order).
        C *vs = lds + (size_t)wave * Q * 64;
#pragma unroll
        for (int k2 = 0; k2 < NVB; ++k2)
            if (lane + 64 * k2 < VB) vs[lane + 64 * k2] = vpf[k2];
        __builtin_amdgcn_wave_barrier();
        C lacc[Q];
#pragma unroll
        for (int i = 0; i < Q; ++i) {
            C acc = czero<C>();
#pragma unroll
            for (int t = 0; t < kLeafPts; ++t) {
                if constexpr (ADJ)
                    cfmac(acc, vs[t * Q + i], x[t]);
                else
                    cfma(acc, vs[i * kLeafPts + t], x[t]);
            }
            lacc[i] = acc;
        }
        __builtin_amdgcn_wave_barrier();
#pragma unroll
        for (int i = 0; i < Q; ++i) lds[(wave * Q + i) * 64 + lane] = lacc[i];
    } else {
        const int lp = wave;
        const long gp = ADJ ? (A * P + lp) * Glast + S : A * 2 * a.G0 + S * P + lp;
        const C *src = a.in + (size_t)gp * Q * ld + (act ? col : (int)blockIdx.y * 64);
        C v[Q];
#pragma unroll
        for (int i = 0; i < Q; ++i) v[i] = src[i * ld];
        if (TWL && tid < NTW) stw[tid] = tw0;
#pragma unroll
        for (int i = 0; i < Q; ++i) lds[(lp * Q + i) * 64 + lane] = act ? v[i] : czero<C>();
    }
    __syncthreads();
    const int grp = wave >> 1, h = wave & 1;
#pragma unroll
    for (int st = 0; st < KL; ++st) {
        const int j = ADJ ? KL - 1 - st : st;
        if (TWL && st + 1 < KL) twn = tw_src(ADJ ? j - 1 : j + 1, tid < NTW ? tid : 0);
        if constexpr (EPI_M && !EARLY_M)
            if (st == KL - 1) fetch_m();
        C acc[Q];
        const int dst = struct_step<T, Q, KL, ADJ, CS>(a, lds, stw + grp * 8 * Q, grp, h, j, lane, acc);
        __syncthreads();
#pragma unroll
        for (int r = 0; r < Q; ++r) lds[(dst * Q + r) * 64 + lane] = acc[r];
        if (TWL && st + 1 < KL && tid < NTW) stw[tid] = twn;
        // After the last factor every wave touches only its own pair's rows (its output pair is
        // its store pair: 2g + h), and LDS runs one wave's accesses in order: no barrier there.
        if (st + 1 < KL) __syncthreads();
    }
    {
        const int lp = wave;
        const long gp = ADJ ? A * 2 * a.G0 + S * P + lp : (A * P + lp) * Glast + S;
        C *dstp = a.out + (size_t)gp * Q * ld + col;
        if (EPI_M) {
            C x[Q];
#pragma unroll
            for (int i = 0; i < Q; ++i) x[i] = lds[(lp * Q + i) * 64 + lane];
            // the pair's rows of the tile are this wave's alone now: the prefetched middle block
            // goes there and is read back as broadcasts
            __builtin_amdgcn_wave_barrier();
            C *mst = lds + (size_t)lp * Q * 64;
#pragma unroll
            for (int k2 = 0; k2 < NMP; ++k2)
                if (lane + 64 * k2 < Q * Q) mst[lane + 64 * k2] = mpf[k2];
            __builtin_amdgcn_wave_barrier();
            const C *m = mst;
#pragma unroll
            for (int i = 0; i < Q; ++i) {
                C acc = czero<C>();
#pragma unroll
                for (int jj = 0; jj < Q; ++jj) {
                    if (ADJ)
                        cfmac(acc, m[jj * Q + i], x[jj]);
                    else
                        cfma(acc, m[i * Q + jj], x[jj]);
                }
                if (act) dstp[i * ld] = acc;
            }
        } else {
#pragma unroll
            for (int i = 0; i < Q; ++i)
                if (act) dstp[i * ld] = lds[(lp * Q + i) * 64 + lane];
        }
    }
}

template <typename T, int Q, int KL, bool CS>
static void launch_struct_cs(const StructArgs<T, Q> &sa, bool adj, bool epi, dim3 grid, dim3 block, hipStream_t s) {
    if (adj) {
        if (epi)
            k_struct_fused<T, Q, KL, true, true, CS><<<grid, block, 0, s>>>(sa);
        else
            k_struct_fused<T, Q, KL, true, false, CS><<<grid, block, 0, s>>>(sa);
    } else {
        if (epi)
            k_struct_fused<T, Q, KL, false, true, CS><<<grid, block, 0, s>>>(sa);
        else
            k_struct_fused<T, Q, KL, false, false, CS><<<grid, block, 0, s>>>(sa);
    }
}

template <typename T, int Q, int KL>
static void launch_struct(const StructArgs<T, Q> &sa, bool adj, bool epi, long N, hipStream_t s) {
    dim3 grid((unsigned)(N >> KL), (unsigned)((sa.nrhs + 63) / 64));
    dim3 block((1 << KL) * 64);
    if (sa.cside)
        launch_struct_cs<T, Q, KL, true>(sa, adj, epi, grid, block, s);
    else
        launch_struct_cs<T, Q, KL, false>(sa, adj, epi, grid, block, s);
}

// The leaf factor folds into a 3-level pass when the pass's tile (8 q coefficient rows of
// 64 columns) can hold the 64 staged input rows of its 64 columns.
template <typename T, int Q> constexpr bool leaf_foldable() { return fused_max_kl<T, Q>() >= 3 && 8 * Q >= 65; }

// The first pass of 3 levels with the leaf factor folded in (k_struct_fused, LEAF): forward
// C side or adjoint B side.
template <typename T, int Q>
static void run_struct_leaf(const StructArgs<T, Q> &sa, bool adj, bool epi, long N, hipStream_t s) {
    if constexpr (leaf_foldable<T, Q>()) {
        const dim3 grid((unsigned)(N >> 3), (unsigned)((sa.nrhs + 63) / 64)), block(8 * 64);
        if (adj) {
            if (epi)
                k_struct_fused<T, Q, 3, true, true, false, true><<<grid, block, 0, s>>>(sa);
            else
                k_struct_fused<T, Q, 3, true, false, false, true><<<grid, block, 0, s>>>(sa);
        } else if (epi) {
            k_struct_fused<T, Q, 3, false, true, true, true><<<grid, block, 0, s>>>(sa);
        } else {
            k_struct_fused<T, Q, 3, false, false, true, true><<<grid, block, 0, s>>>(sa);
        }
    } else {
        throw Err{FIO_ERR_UNSUPPORTED};
    }
}

template <typename T, int Q>
static void run_struct(const StructArgs<T, Q> &sa, int kl, bool adj, bool epi, long N, hipStream_t s) {
    switch (kl) {
        case 1: launch_struct<T, Q, 1>(sa, adj, epi, N, s); break;
        case 2: launch_struct<T, Q, 2>(sa, adj, epi, N, s); break;
        case 3:
            if constexpr (fused_max_kl<T, Q>() >= 3) {
                launch_struct<T, Q, 3>(sa, adj, epi, N, s);
                break;
            }
            [[fallthrough]];
        default: throw Err{FIO_ERR_UNSUPPORTED};
    }
}


// Leaf factors with coalesced block I/O.  A workgroup (256 threads) owns 4 leaf boxes
// (32 consecutive rows of the N x nrhs block) and 64 right-hand sides.  The block is
// moved between HBM and LDS with lanes along rows (coalesced in the column-major
// layout) and used with lanes along columns, as the coefficient buffers are.
//   IN  = true : coefficients of the 8 boxes x 8 coarse partners from the vector
//                (V forward, U^* adjoint);
//   IN  = false: the vector from the coefficients (U forward, V^* adjoint).
// Coarse partner c of leaf box b has pair index b nsl + c (U side) or c 2^L' + b (V side).
template <typename T, int Q, bool IN, bool VSIDE>
__global__ void __launch_bounds__(256, 4) k_leaf_io(Geo g, const cpx<T> *__restrict__ Fblk,
                                                 const double2 *__restrict__ Xin, long ldx,
                                                 const cpx<T> *__restrict__ cin, cpx<T> *__restrict__ cout,
                                                 double2 *__restrict__ Yout, long ldy, int nrhs,
                                                 const double2 *__restrict__ Ysub, long ldsub) {
    using C = cpx<T>;
    constexpr int NB = 4;                           // leaf boxes per workgroup
    constexpr int R = NB * kLeafPts;                // rows per workgroup
    constexpr int BLK = Q * kLeafPts;               // complex entries of one factor block
    constexpr int NCH = BLK * (int)sizeof(C) / 16;  // its 16-byte chunks
    constexpr int NPF = (NCH + 63) / 64;
    __shared__ C tile[64][R + 1];                   // [column][row]
    // one factor block per wave; the block of the wave's next unit (IN) or next coarse partner
    // (out) is fetched into registers (vector loads) while the current one is applied, then
    // written here and read back as broadcasts
    __shared__ __attribute__((aligned(16))) C wblk[4][BLK];
    const int tid = threadIdx.x, lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const long box0 = (long)blockIdx.x * NB;        // first leaf box of the workgroup
    const int c0 = blockIdx.y * 64;
    const int ncol = nrhs - c0 < 64 ? nrhs - c0 : 64;
    const int col = c0 + lane;
    const bool act = lane < ncol;
    const long Lp2 = 1L << g.Lp;
    // V[sigma = box][tau = c] and U[tau = box][sigma = c] both sit at (box nsl + c) BLK
    uint4 pf[NPF];
    auto fetch = [&](long box, int c) {
        const uint4 *src = reinterpret_cast<const uint4 *>(Fblk + ((size_t)box * g.nsl + c) * BLK);
#pragma unroll
        for (int k = 0; k < NPF; ++k)
            if (lane + 64 * k < NCH) pf[k] = src[lane + 64 * k];
    };
    auto stage = [&]() {
        uint4 *dst = reinterpret_cast<uint4 *>(&wblk[wave][0]);
#pragma unroll
        for (int k = 0; k < NPF; ++k)
            if (lane + 64 * k < NCH) dst[lane + 64 * k] = pf[k];
    };
    if (IN) {
        const C *blk = &wblk[wave][0];
        if (wave < NB * g.nsl) {
            fetch(box0 + wave / g.nsl, wave % g.nsl);
            stage();
        }
        for (int e = tid; e < R * 64; e += 256) {
            const int r = e % R, cc = e / R;
            double2 v = cc < ncol ? Xin[(box0 * kLeafPts + r) + (size_t)(c0 + cc) * ldx] : zc(0.0, 0.0);
            tile[cc][r] = cmake<C>((T)v.x, (T)v.y);
        }
        __syncthreads();
        // unit = (local box b, coarse partner c)
        for (int u = wave; u < NB * g.nsl; u += 4) {
            const int b = u / g.nsl, c = u % g.nsl;
            const long box = box0 + b;
            const int un = u + 4;
            if (un < NB * g.nsl) fetch(box0 + un / g.nsl, un % g.nsl);
            C x[kLeafPts];
#pragma unroll
            for (int s = 0; s < kLeafPts; ++s) x[s] = tile[lane][b * kLeafPts + s];
            // V: block (q x 8) for pair c 2^L' + box; U^*: block (8 x q) for pair box nsl + c
            const size_t p = VSIDE ? (size_t)c * Lp2 + box : (size_t)box * g.nsl + c;
            C *op = cout + p * Q * (size_t)nrhs + col;
#pragma unroll
            for (int j = 0; j < Q; ++j) {
                C acc = czero<C>();
#pragma unroll
                for (int s = 0; s < kLeafPts; ++s) {
                    if (VSIDE)
                        cfma(acc, blk[j * kLeafPts + s], x[s]);
                    else
                        cfmac(acc, blk[s * Q + j], x[s]);
                }
                if (act) op[(size_t)j * nrhs] = acc;
            }
            // the wave's reads of this block precede the overwrite (LDS runs a wave's accesses in order)
            __builtin_amdgcn_wave_barrier();
            if (un < NB * g.nsl) stage();
            __builtin_amdgcn_wave_barrier();
        }
    } else {
        // each wave produces one box's rows for its lane's column (NB = 4 boxes, 4 waves)
        static_assert(NB == 4, "one leaf box per wave");
        const int b = wave;
        const long box = box0 + b;
        const C *blk = &wblk[wave][0];
        C acc[kLeafPts];
#pragma unroll
        for (int s = 0; s < kLeafPts; ++s) acc[s] = czero<C>();
        // blocks of partners c = 0 .. nsl - 1 of the box follow one another in memory
        const uint4 *bsrc = reinterpret_cast<const uint4 *>(Fblk + (size_t)box * g.nsl * BLK);
        uint4 *bdst = reinterpret_cast<uint4 *>(&wblk[wave][0]);
#pragma unroll
        for (int k = 0; k < NPF; ++k)
            if (lane + 64 * k < NCH) bdst[lane + 64 * k] = bsrc[lane + 64 * k];
        __builtin_amdgcn_wave_barrier();
        for (int c = 0; c < g.nsl; ++c) {
            // V^*: block V[sigma = box][tau = c], pair c 2^L' + box; U: block U[tau = box][sigma = c],
            // pair box nsl + c.  The next partner's block is on its way while this one is applied.
            const size_t p = VSIDE ? (size_t)c * Lp2 + box : (size_t)box * g.nsl + c;
            uint4 nb[NPF];
            const bool more = c + 1 < g.nsl;
#pragma unroll
            for (int k = 0; k < NPF; ++k)
                if (more && lane + 64 * k < NCH) nb[k] = bsrc[(size_t)(c + 1) * NCH + lane + 64 * k];
            // inactive lanes (columns beyond nrhs) read column c0 and use zeros: no branches
            C d[Q];
            const C *ip = cin + p * Q * (size_t)nrhs + (act ? col : c0);
#pragma unroll
            for (int i = 0; i < Q; ++i) {
                const C v = ip[(size_t)i * nrhs];
                d[i] = act ? v : czero<C>();
            }
            // input index outermost (each acc[s] still sums over i in order): one column of the
            // block is live at a time
#pragma unroll
            for (int i = 0; i < Q; ++i) {
#pragma unroll
                for (int s = 0; s < kLeafPts; ++s) {
                    if (VSIDE)
                        cfmac(acc[s], blk[i * kLeafPts + s], d[i]);
                    else
                        cfma(acc[s], blk[s * Q + i], d[i]);
                }
            }
            // The products are finished before the next block overwrites this one (else the
            // compiler would read the whole block ahead, hold it in vector registers and sink the
            // products below the overwrite); LDS runs a wave's accesses in order.
#pragma unroll
            for (int s = 0; s < kLeafPts; ++s) asm volatile("" : "+v"(acc[s].x), "+v"(acc[s].y)::"memory");
            __builtin_amdgcn_wave_barrier();
#pragma unroll
            for (int k = 0; k < NPF; ++k)
                if (more && lane + 64 * k < NCH) bdst[lane + 64 * k] = nb[k];
            __builtin_amdgcn_wave_barrier();
        }
#pragma unroll
        for (int s = 0; s < kLeafPts; ++s) tile[lane][b * kLeafPts + s] = acc[s];
        __syncthreads();
        for (int e = tid; e < R * 64; e += 256) {
            const int r = e % R, cc = e / R;
            if (cc < ncol) {
                C v = tile[cc][r];
                double2 y = zc((double)v.x, (double)v.y);
                if (Ysub) {
                    // Yout = Ysub - (the apply), the residual of a refinement step
                    const double2 u = Ysub[(box0 * kLeafPts + r) + (size_t)(c0 + cc) * ldsub];
                    y = zc(u.x - y.x, u.y - y.y);
                }
                Yout[(box0 * kLeafPts + r) + (size_t)(c0 + cc) * ldy] = y;
            }
        }
    }
}

template <typename T, int Q>
static void apply_q(fio_bf_s *bf, bool adj, const double2 *X, long ldx, double2 *Y, long ldy, int nrhs,
                    const cpx<T> *F, cpx<T> *c0, cpx<T> *c1, hipStream_t s, bool split, const double2 *Ysub,
                    long ldsub) {
    Geo g = geo_of(bf);
    const unsigned TB = 256;
    const bool uni = (nrhs % 64) == 0;
    const size_t nleaf = (size_t)(1L << bf->Lp) * bf->nsl;
    const long ng = bf->N / 2, np = bf->N;
    cpx<T> *cur = c0, *nxt = c1;
    const bool f64 = sizeof(T) == 8;
    auto transfer = [&](size_t off, long G, bool a) {
        size_t nt = (size_t)ng * nrhs;
        FIO_TIMED(f64 ? "bf_transfer_f64" : "bf_transfer_f32", s);
        if (a) {
            if (uni)
                k_transfer<T, Q, true, true><<<grid1d(nt, TB), TB, 0, s>>>(F + off, G, cur, nxt, ng, nrhs);
            else
                k_transfer<T, Q, true, false><<<grid1d(nt, TB), TB, 0, s>>>(F + off, G, cur, nxt, ng, nrhs);
        } else {
            if (uni)
                k_transfer<T, Q, false, true><<<grid1d(nt, TB), TB, 0, s>>>(F + off, G, cur, nxt, ng, nrhs);
            else
                k_transfer<T, Q, false, false><<<grid1d(nt, TB), TB, 0, s>>>(F + off, G, cur, nxt, ng, nrhs);
        }
        std::swap(cur, nxt);
    };
    // fused passes: levels [lo, hi) of the C side (cside) or the B side; forward C passes
    // run C^[h+hi] .. C^[h+lo+1], forward B passes run B^[h+lo+1] .. B^[h+hi]
    bool fused = false;
    int kmax = 1;
    bool leaf_sep = false;
    if constexpr (fused_q<Q>()) {
        fused = bf->nl > 0 && (split || !fused_disabled());
        kmax = fused_max_kl<T, Q>();
        // levels per pass: tuned (fio_bf_autotune) or the most the LDS tile holds; the tuned
        // configuration may also keep the first leaf factor separate and, in split precision,
        // run the transfer passes on the vector units in FP32
        const fio_prec pr = f64 ? FIO_PREC_FP64 : (split ? FIO_PREC_SPLIT_FP16 : FIO_PREC_FP32);
        const TileCfg tc = bf_tile(bf, adj, pr, nrhs);
        if (tc.kmax > 0 && tc.kmax < kmax) kmax = tc.kmax;
        leaf_sep = tc.leaf_sep != 0;
        if (split && tc.valu) split = false;
    }
    auto pass = [&](bool a, bool cside, int lo, int hi, bool epi, bool leaf = false) {
        if constexpr (fused_q<Q>()) {
            const int kl = hi - lo;
            if constexpr (std::is_same<T, float>::value && Q == 9) {
                // split FP16 runs every pass on the matrix cores except a first pass with the
                // leaf factor folded in, which runs as the FP32 structured pass (same coefficient
                // layout, more precise; saves the separate leaf kernel)
                if (split && !leaf) {
                    SplitPass sp;
                    for (int jj = 0; jj < 3; ++jj) sp.A[jj] = nullptr;
                    for (int jj = 0; jj < kl; ++jj)
                        sp.A[jj] = split_blocks(bf, cside, cside ? hi - 1 - jj : lo + jj, a);
                    sp.G0 = cside ? (1L << (bf->h + hi - 1)) : (1L << (bf->L - (bf->h + lo) - 1));
                    sp.in = cur;
                    sp.out = nxt;
                    sp.nrhs = nrhs;
                    FIO_TIMED("bf_split16", s);
                    // the middle factor is folded into the split blocks next to it
                    split_pass(sp, kl, a, bf->N, s);
                    std::swap(cur, nxt);
                    return;
                }
            }
            if (bf->structured) {
                StructArgs<T, Q> sa;
                const cpx<T> *TWb = f64 ? reinterpret_cast<const cpx<T> *>(bf->tw64.p)
                                        : reinterpret_cast<const cpx<T> *>(bf->tw32.p);
                for (int jj = 0; jj < 4; ++jj) sa.TW[jj] = nullptr;
                for (int jj = 0; jj < kl; ++jj)
                    sa.TW[jj] = TWb + bf_tw_off(bf, cside, cside ? hi - 1 - jj : lo + jj);
                sa.M = F + bf->offM;
                sa.G0 = cside ? (1L << (bf->h + hi - 1)) : (1L << (bf->L - (bf->h + lo) - 1));
                sa.in = cur;
                sa.out = nxt;
                sa.nrhs = nrhs;
                sa.cside = cside ? 1 : 0;
                sa.V = F + (a ? bf->offU : bf->offV);
                sa.X = X;
                sa.ldx = ldx;
                for (int c = 0; c < 2; ++c)
                    for (int i = 0; i < Q; ++i)
                        for (int t = 0; t < Q; ++t) {
                            sa.P[c][i][t] = (T)bf->Pchild[(c * Q + i) * Q + t];
                            sa.PT[c][t][i] = sa.P[c][i][t];
                        }
                // symmetric and antisymmetric row combinations of G_0 = P_0^T, in double
                // precision before rounding to T: G_0(r, t) = P_0(t, r)
                for (int t = 0; t < Q; ++t) {
                    const double *p0 = bf->Pchild;
                    for (int r = 0; r < (Q + 1) / 2; ++r) {
                        const double g = p0[t * Q + r], gm = p0[t * Q + (Q - 1 - r)];
                        sa.SD[t][r] = (T)(2 * r + 1 == Q ? g : 0.5 * (g + gm));
                    }
                    for (int r = 0; r < Q / 2; ++r) {
                        const double g = p0[t * Q + r], gm = p0[t * Q + (Q - 1 - r)];
                        sa.SD[t][(Q + 1) / 2 + r] = (T)(0.5 * (g - gm));
                    }
                }
                if (leaf) {
                    FIO_TIMED(f64 ? "bf_struct_leaf_f64" : "bf_struct_leaf_f32", s);
                    run_struct_leaf<T, Q>(sa, a, epi, bf->N, s);
                } else {
                    FIO_TIMED(f64 ? "bf_struct_f64" : "bf_struct_f32", s);
                    run_struct<T, Q>(sa, kl, a, epi, bf->N, s);
                }
                std::swap(cur, nxt);
                return;
            }
            FusedArgs<T> fa;
            for (int j = 0; j < 4; ++j) fa.A[j] = nullptr;
            for (int j = 0; j < kl; ++j)
                fa.A[j] = F + (cside ? bf->offC[hi - 1 - j] : bf->offB[lo + j]);
            fa.M = F + bf->offM;
            fa.G0 = cside ? (1L << (bf->h + hi - 1)) : (1L << (bf->L - (bf->h + lo) - 1));
            fa.in = cur;
            fa.out = nxt;
            fa.nrhs = nrhs;
            fa.sink = 0;
            fa.sink_ptr = reinterpret_cast<double *>(nxt);
            FIO_TIMED(f64 ? "bf_fused_f64" : "bf_fused_f32", s);
            run_fused<T, Q>(fa, kl, a, epi, bf->N, s);
            std::swap(cur, nxt);
        }
    };
    auto middle = [&](bool a) {
        size_t nt = (size_t)np * nrhs;
        FIO_TIMED(f64 ? "bf_middle_f64" : "bf_middle_f32", s);
        if (a) {
            if (uni)
                k_middle<T, Q, true, true><<<grid1d(nt, TB), TB, 0, s>>>(F + bf->offM, cur, nxt, np, nrhs);
            else
                k_middle<T, Q, true, false><<<grid1d(nt, TB), TB, 0, s>>>(F + bf->offM, cur, nxt, np, nrhs);
        } else {
            if (uni)
                k_middle<T, Q, false, true><<<grid1d(nt, TB), TB, 0, s>>>(F + bf->offM, cur, nxt, np, nrhs);
            else
                k_middle<T, Q, false, false><<<grid1d(nt, TB), TB, 0, s>>>(F + bf->offM, cur, nxt, np, nrhs);
        }
        std::swap(cur, nxt);
    };
    const bool tiled = ((1L << bf->Lp) % 4) == 0;
    const dim3 tgrid((unsigned)((1L << bf->Lp) / 4), (unsigned)((nrhs + 63) / 64));
    if (!adj) {
        // V^[L'] folds into the first C pass when that pass is a structured one of 3 levels (one
        // leaf box per wave) and its workgroups can be grouped by 8 per XCD (2^L' / 8 % 8 == 0)
        const bool leaf_fused = leaf_foldable<T, Q>() && fused && bf->structured &&
                                !leaf_fused_disabled() && !leaf_sep && (kmax < bf->nl ? kmax : bf->nl) == 3 &&
                                bf->Lp >= 6;
        if (!leaf_fused) {
            FIO_TIMED(f64 ? "bf_leaf_in_f64" : "bf_leaf_in_f32", s);
            if (tiled)
                k_leaf_io<T, Q, true, true><<<tgrid, 256, 0, s>>>(g, F + bf->offV, X, ldx, nullptr, cur, nullptr, 0,
                                                                  nrhs, nullptr, 0);
            else
                k_leaf_in_fwd<T, Q><<<grid1d(nleaf * nrhs, TB), TB, 0, s>>>(g, F + bf->offV, X, ldx, cur, nrhs);
        }
        if (fused) {
            // C^[L'] .. C^[h+1] in passes from the top; the last pass also applies M
            for (int hi = bf->nl; hi > 0;) {
                const int lo = hi - kmax > 0 ? hi - kmax : 0;
                pass(false, true, lo, hi, lo == 0, leaf_fused && hi == bf->nl);
                hi = lo;
            }
            for (int lo = 0; lo < bf->nl;) {
                const int hi = lo + kmax < bf->nl ? lo + kmax : bf->nl;
                pass(false, false, lo, hi, false);
                lo = hi;
            }
        } else {
            for (int lev = bf->nl - 1; lev >= 0; --lev) transfer(bf->offC[lev], 1L << (bf->h + lev), false);
            middle(false);
            for (int lev = 0; lev < bf->nl; ++lev) transfer(bf->offB[lev], 1L << (bf->L - bf->h - lev - 1), false);
        }
        FIO_TIMED(f64 ? "bf_leaf_out_f64" : "bf_leaf_out_f32", s);
        if (tiled)
            k_leaf_io<T, Q, false, false><<<tgrid, 256, 0, s>>>(g, F + bf->offU, nullptr, 0, cur, nullptr, Y, ldy,
                                                                nrhs, Ysub, ldsub);
        else
            k_leaf_out_fwd<T, Q><<<grid1d(((size_t)1 << bf->Lp) * nrhs, TB), TB, 0, s>>>(g, F + bf->offU, cur, Y,
                                                                                           ldy, nrhs, Ysub, ldsub);
    } else {
        // U^[L']* folds into the first B* pass under the same conditions as V^[L'] forward
        const bool leaf_fused = leaf_foldable<T, Q>() && fused && bf->structured &&
                                !leaf_fused_disabled() && !leaf_sep && (kmax < bf->nl ? kmax : bf->nl) == 3 &&
                                bf->Lp >= 6;
        if (!leaf_fused) {
            FIO_TIMED(f64 ? "bf_leaf_in_f64" : "bf_leaf_in_f32", s);
            if (tiled)
                k_leaf_io<T, Q, true, false><<<tgrid, 256, 0, s>>>(g, F + bf->offU, X, ldx, nullptr, cur, nullptr, 0,
                                                                   nrhs, nullptr, 0);
            else
                k_leaf_in_adj<T, Q><<<grid1d(nleaf * nrhs, TB), TB, 0, s>>>(g, F + bf->offU, X, ldx, cur, nrhs);
        }
        if (fused) {
            // B^[L']* .. B^[h+1]* in passes from the top; the last pass also applies M*
            for (int hi = bf->nl; hi > 0;) {
                const int lo = hi - kmax > 0 ? hi - kmax : 0;
                pass(true, false, lo, hi, lo == 0, leaf_fused && hi == bf->nl);
                hi = lo;
            }
            for (int lo = 0; lo < bf->nl;) {
                const int hi = lo + kmax < bf->nl ? lo + kmax : bf->nl;
                pass(true, true, lo, hi, false);
                lo = hi;
            }
        } else {
            for (int lev = bf->nl - 1; lev >= 0; --lev) transfer(bf->offB[lev], 1L << (bf->L - bf->h - lev - 1), true);
            middle(true);
            for (int lev = 0; lev < bf->nl; ++lev) transfer(bf->offC[lev], 1L << (bf->h + lev), true);
        }
        FIO_TIMED(f64 ? "bf_leaf_out_f64" : "bf_leaf_out_f32", s);
        if (tiled)
            k_leaf_io<T, Q, false, true><<<tgrid, 256, 0, s>>>(g, F + bf->offV, nullptr, 0, cur, nullptr, Y, ldy,
                                                               nrhs, nullptr, 0);
        else
            k_leaf_out_adj<T, Q><<<grid1d(((size_t)1 << bf->Lp) * nrhs, TB), TB, 0, s>>>(g, F + bf->offV, cur, Y,
                                                                                           ldy, nrhs);
    }
    FIO_HIP(hipGetLastError());
}

template <typename T>
void apply_t(fio_bf_s *bf, bool adj, const double2 *X, long ldx, double2 *Y, long ldy, int nrhs,
                    const cpx<T> *F, void *ws, hipStream_t s, bool split = false, const double2 *Ysub = nullptr,
                    long ldsub = 0) {
    cpx<T> *c0 = reinterpret_cast<cpx<T> *>(ws);
    cpx<T> *c1 = c0 + bf_coef_elems(bf, nrhs);
    switch (bf->q) {
#define FIO_Q(QQ) \
    case QQ: apply_q<T, QQ>(bf, adj, X, ldx, Y, ldy, nrhs, F, c0, c1, s, split, Ysub, ldsub); break;
        FIO_Q(2) FIO_Q(3) FIO_Q(4) FIO_Q(5) FIO_Q(6) FIO_Q(7) FIO_Q(8) FIO_Q(9)
        FIO_Q(10) FIO_Q(11) FIO_Q(12) FIO_Q(13) FIO_Q(14) FIO_Q(15) FIO_Q(16)
#undef FIO_Q
        default: throw Err{FIO_ERR_UNSUPPORTED};
    }
}

}  // namespace fio
