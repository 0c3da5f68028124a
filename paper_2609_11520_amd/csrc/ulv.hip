// ULV factorization of an HPD HSS matrix and its solve (Section 2.4) on gfx950.
//
// Factor (offline, one workgroup per node, level by level from the leaves):
//   QL basis elimination U = Q [0; Uhat2] with Householder reflectors taken from
//   the bottom of each column; Dchk = Q^* D Q; Cholesky Dchk11 = L11 L11^*;
//   Dhat21 = Dchk21 L11^{-*}; Dhat22 = Dchk22 - Dhat21 Dhat21^*; then the merge
//   of eq. ulv_merge for every parent and a Cholesky of the root block.
// The two solve sweeps of Section 2.4 are stored per node as one m x m matrix
//   W = [L11^{-1} Q1^*; Q2^* - Dhat21 L11^{-1} Q1^*]
// so that the bottom-up step is [bhat1; yhat2] = W y_tau and the top-down step is
// c_tau = W^* [bhat1; chat2]; the root keeps Linv = L_rho^{-1}.  The online solve
// is therefore 2 Lh + 2 batched small GEMM launches (see k_ulv_level).
#include "hss.h"
#include "timing.h"

#include <cmath>
#include <cstring>

struct hss_ulv_s {
    long N = 0;
    int leaf = 0, Lh = 0, m0 = 0;
    std::vector<std::vector<int>> m, k, r;      // per level (1..Lh)
    std::vector<std::vector<size_t>> woff;
    std::vector<std::vector<long>> yoff, roff;  // rows of a node in its level vector / parent vector
    std::vector<long> rows;                     // rows of the level-l vector (l = 0..Lh)
    fio::DevBuf W;                              // all W slots
    fio::DevBuf WH;                             // W^* of every node (same offsets), for narrow solves
    fio::DevBuf Linv;                           // m0 x m0
    fio::DevBuf meta;                           // device copies of the per-level tables
    std::vector<size_t> meta_woff, meta_m, meta_k, meta_yoff, meta_roff;   // byte offsets into meta
    fio::DevBuf rootdesc;                       // ZgemmDesc[2] for the root (pointers into ws set per call)
    fio::DevBuf ws;
    std::mutex ws_mu;
};

namespace fio {

constexpr int kUlvMaxM = 2048;   // largest node size of the factorization
// one workgroup per node; large nodes (upper levels of 2D trees) get 16 waves
inline unsigned ulv_threads(int m) { return m >= 192 ? 1024u : 256u; }

__device__ __forceinline__ double wsum(double v, double *sh) {
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    __syncthreads();
    if (lane == 0) sh[w] = v;
    __syncthreads();
    double t = 0.0;
    for (int i = 0; i < (int)(blockDim.x >> 6); ++i) t += sh[i];
    return t;
}

// In-place Cholesky (lower) of the leading n x n block of A (column-major, lda).
// Returns false (on every thread) when a pivot is not positive.
__device__ bool wg_potrf(double2 *A, int lda, int n, double *sh, int *s_flag) {
    const int tid = threadIdx.x, nt = blockDim.x;
    if (tid == 0) *s_flag = 0;
    __syncthreads();
    for (int c = 0; c < n; ++c) {
        double d = A[c + (size_t)c * lda].x;
        if (!(d > 0.0) || !isfinite(d)) {
            if (tid == 0) *s_flag = 1;
            __syncthreads();
            return false;
        }
        d = sqrt(d);
        __syncthreads();
        for (int i = c + tid; i < n; i += nt) {
            double2 v = A[i + (size_t)c * lda];
            A[i + (size_t)c * lda] = i == c ? zc(d, 0.0) : zc(v.x / d, v.y / d);
        }
        __syncthreads();
        // trailing update of the lower triangle: A(i, j) -= L(i, c) conj(L(j, c)), c < j <= i
        const int rem = n - c - 1;
        for (int e = tid; e < rem * rem; e += nt) {
            int i = c + 1 + e % rem, j = c + 1 + e / rem;
            if (j > i) continue;
            double2 li = A[i + (size_t)c * lda], lj = A[j + (size_t)c * lda];
            double2 &a = A[i + (size_t)j * lda];
            a.x -= li.x * lj.x + li.y * lj.y;
            a.y -= li.y * lj.x - li.x * lj.y;
        }
        __syncthreads();
    }
    // clear the strict upper triangle (not part of L)
    for (int e = tid; e < n * n; e += nt) {
        int i = e % n, j = e / n;
        if (j > i) A[i + (size_t)j * lda] = zc(0.0, 0.0);
    }
    __syncthreads();
    (void)sh;
    return true;
}

struct FactArgs {
    // inputs per node of the level
    const double2 *D;       // node diagonal blocks
    const size_t *doff;
    const double2 *U;       // node bases
    const size_t *uoff;
    const int *msz, *rsz;
    // outputs
    double2 *W;             // m x m per node
    const size_t *woff;
    double2 *D22;           // r x r per node (slot m x m)
    double2 *U2;            // r x r per node (slot m x m)
    const size_t *soff;
    double2 *scratch;       // 3 m^2 per node
    const size_t *scoff;
    int *fail;
};

// Basis elimination, partial Cholesky and the node's W (one workgroup per node), in two
// phases around the two dense products Dchk = Q^* D Q, which run as batched GEMMs over
// all nodes of the level:
//   PHASE 0: QL of U_tau (Householder), explicit Q, the reduced basis U2;
//   PHASE 1: Cholesky of Dchk11, Dhat21, Dhat22 and W = [L11^{-1} Q1^*; Q2^* - Dhat21 L11^{-1} Q1^*].
template <int PHASE>
__global__ void __launch_bounds__(1024) k_ulv_node(FactArgs a) {
    __shared__ double sh[16];
    __shared__ double s_tau[kUlvMaxM];
    __shared__ int s_flag;
    const int node = blockIdx.x, tid = threadIdx.x, nt = blockDim.x;
    const int m = a.msz[node], r = a.rsz[node], k = m - r;
    if (m == 0) return;
    double2 *Uw = a.scratch + a.scoff[node];        // m x r working copy, then reflectors
    double2 *Q = Uw + (size_t)m * m;                 // m x m explicit Q
    double2 *T = Q + (size_t)m * m;                  // m x m: Dchk = Q^* D Q (batched GEMMs)
    const double2 *Uin = a.U + a.uoff[node];
    double2 *Wm = a.W + a.woff[node];
    if constexpr (PHASE == 0) {
        for (int e = tid; e < m * r; e += nt) Uw[e] = Uin[e];
        __syncthreads();
        // QL: for column jj = r-1..0 eliminate rows 0..p-1 (p = k + jj) into row p
        for (int jj = r - 1; jj >= 0; --jj) {
            const int p = k + jj, n = p + 1;
            double2 *x = Uw + (size_t)jj * m;            // rows 0..p
            const double2 al = x[p];
            double part = 0.0;
            for (int i = tid; i < n; i += nt) part += x[i].x * x[i].x + x[i].y * x[i].y;
            const double sigma = sqrt(wsum(part, sh));
            double tau = 0.0;
            if (sigma > 0.0) {
                const double aa = sqrt(al.x * al.x + al.y * al.y);
                double2 ph = aa > 0.0 ? zc(al.x / aa, al.y / aa) : zc(1.0, 0.0);
                double2 beta = zc(-ph.x * sigma, -ph.y * sigma);
                double2 den = csub(al, beta);
                double dn = den.x * den.x + den.y * den.y;
                double2 inv = zc(den.x / dn, -den.y / dn);
                for (int i = tid; i < p; i += nt) x[i] = cmul(x[i], inv);
                __syncthreads();
                if (tid == 0) x[p] = beta;
                tau = 1.0 + aa / sigma;
            }
            if (tid == 0) s_tau[jj] = tau;
            __syncthreads();
            // apply H = I - tau v v^*, v = [x[0..p); 1], to columns 0..jj-1 (rows 0..p)
            if (tau != 0.0) {
                for (int c = tid; c < jj; c += nt) {
                    double2 *col = Uw + (size_t)c * m;
                    double2 w = col[p];
                    for (int i = 0; i < p; ++i) cfmac(w, x[i], col[i]);
                    double2 tw = zc(tau * w.x, tau * w.y);
                    col[p] = csub(col[p], tw);
                    for (int i = 0; i < p; ++i) col[i] = csub(col[i], cmul(x[i], tw));
                }
            }
            __syncthreads();
        }
        // Q = H_{r-1} ... H_0 I: apply H_0 first
        for (int e = tid; e < m * m; e += nt) Q[e] = zc((e % m) == (e / m) ? 1.0 : 0.0, 0.0);
        __syncthreads();
        for (int jj = 0; jj < r; ++jj) {
            const double tau = s_tau[jj];
            if (tau == 0.0) continue;
            const int p = k + jj;
            const double2 *x = Uw + (size_t)jj * m;
            for (int c = tid; c < m; c += nt) {
                double2 *col = Q + (size_t)c * m;
                double2 w = col[p];
                for (int i = 0; i < p; ++i) cfmac(w, x[i], col[i]);
                double2 tw = zc(tau * w.x, tau * w.y);
                col[p] = csub(col[p], tw);
                for (int i = 0; i < p; ++i) col[i] = csub(col[i], cmul(x[i], tw));
            }
            __syncthreads();
        }
        // Uhat2: rows k..m-1 of the transformed U (lower triangular r x r: entries j >= i of the
        // reflector-free part); the transformed U is [0; L] with L(i, c) at row k + i, column c
        double2 *U2 = a.U2 + a.soff[node];
        for (int e = tid; e < r * r; e += nt) {
            int i = e % r, c = e / r;
            U2[e] = (c <= i) ? Uw[(k + i) + (size_t)c * m] : zc(0.0, 0.0);
        }
        return;
    }
    // T holds Dchk = (Q^* D) Q (the W slot held Q^* D); Cholesky of Dchk11 (k x k) in place
    if (!wg_potrf(T, m, k, sh, &s_flag)) {
        if (tid == 0) atomicAdd(a.fail, 1);
        return;
    }
    // X = Dhat21^* = L11^{-1} Dchk12 (k x r; Dchk is Hermitian, so Dchk12 = Dchk21^*), in place
    // in T(0..k, k..m), forward substitution per column
    for (int c = tid; c < r; c += nt) {
        double2 *col = T + (size_t)(k + c) * m;
        for (int i = 0; i < k; ++i) {
            double2 acc = col[i];
            for (int l = 0; l < i; ++l) acc = csub(acc, cmul(T[i + (size_t)l * m], col[l]));
            const double d = T[i + (size_t)i * m].x;
            col[i] = zc(acc.x / d, acc.y / d);
        }
    }
    // Dhat22 starts as Dchk22; the level's batched GEMM subtracts X^* X
    double2 *D22 = a.D22 + a.soff[node];
    for (int e = tid; e < r * r; e += nt) {
        const int i = e % r, j = e / r;
        D22[e] = T[(k + i) + (size_t)(k + j) * m];
    }
    // W1 = L11^{-1} Q1^* (k x m), forward substitution per column c of Q1^*
    for (int c = tid; c < m; c += nt) {
        for (int i = 0; i < k; ++i) {
            double2 q = Q[c + (size_t)i * m];            // Q1^*(i, c) = conj(Q(c, i))
            double2 acc = zc(q.x, -q.y);
            for (int l = 0; l < i; ++l) {
                double2 t = cmul(T[i + (size_t)l * m], Wm[l + (size_t)c * m]);
                acc = csub(acc, t);
            }
            double d = T[i + (size_t)i * m].x;
            Wm[i + (size_t)c * m] = zc(acc.x / d, acc.y / d);
        }
    }
    // W2 starts as Q2^* (r x m); the level's batched GEMM subtracts X^* W1 (= Dhat21 W1)
    for (int e = tid; e < r * m; e += nt) {
        const int i = e % r, c = e / r;
        const double2 q = Q[c + (size_t)(k + i) * m];
        Wm[(k + i) + (size_t)c * m] = zc(q.x, -q.y);
    }
}

// ---------------------------------------------------------------------------
// Large nodes (upper levels of 2D trees): phase 0 of k_ulv_node with one reflector per
// launch spread over many workgroups (grid.y = node, grid.x = 64-column chunk).  Node j of
// the level eliminates its columns jj = r-1 .. 0 at host steps t = r-1-jj, and builds Q
// with jj = t.  Same reflector arithmetic as k_ulv_node; the dot products run over four
// lanes per column.
struct UlvBig {
    FactArgs f;
    double *tau;            // kUlvMaxM per node
};

constexpr int kUlvChunk = 16, kUlvThreads = 4 * kUlvChunk;   // columns per workgroup, four lanes each

__global__ void k_ubig_init(UlvBig b) {
    const FactArgs &a = b.f;
    const int node = blockIdx.y, m = a.msz[node], r = a.rsz[node];
    if (m == 0) return;
    double2 *Uw = a.scratch + a.scoff[node], *Q = Uw + (size_t)m * m;
    const double2 *Uin = a.U + a.uoff[node];
    for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < (long)m * m; e += (long)gridDim.x * blockDim.x) {
        if (e < (long)m * r) Uw[e] = Uin[e];
        Q[e] = zc((e % m) == (e / m) ? 1.0 : 0.0, 0.0);
    }
}

__global__ void __launch_bounds__(1024) k_ubig_house(UlvBig b, int t) {
    __shared__ double sh[16];
    const FactArgs &a = b.f;
    const int node = blockIdx.y, m = a.msz[node], r = a.rsz[node], k = m - r;
    const int jj = r - 1 - t;
    if (m == 0 || jj < 0) return;
    const int tid = threadIdx.x, nt = blockDim.x;
    const int p = k + jj, n = p + 1;
    double2 *x = a.scratch + a.scoff[node] + (size_t)jj * m;
    const double2 al = x[p];
    double part = 0.0;
    for (int i = tid; i < n; i += nt) part += x[i].x * x[i].x + x[i].y * x[i].y;
    const double sigma = sqrt(wsum(part, sh));
    double tau = 0.0;
    if (sigma > 0.0) {
        const double aa = sqrt(al.x * al.x + al.y * al.y);
        const double2 ph = aa > 0.0 ? zc(al.x / aa, al.y / aa) : zc(1.0, 0.0);
        const double2 beta = zc(-ph.x * sigma, -ph.y * sigma);
        const double2 den = csub(al, beta);
        const double dn = den.x * den.x + den.y * den.y;
        const double2 inv = zc(den.x / dn, -den.y / dn);
        for (int i = tid; i < p; i += nt) x[i] = cmul(x[i], inv);
        __syncthreads();
        if (tid == 0) x[p] = beta;
        tau = 1.0 + aa / sigma;
    }
    if (tid == 0) b.tau[(size_t)node * kUlvMaxM + jj] = tau;
}

// columns [c0, c1) of A (lda) <- H A, H = I - tau v v^*, v = [x[0..p); 1] (rows 0..p)
__device__ void ql_apply_cols(const double2 *x, int p, double tau, double2 *A, int lda, int c0, int c1) {
    const int sub = threadIdx.x & 3;
    for (int cb = c0; cb < c1; cb += (int)(blockDim.x >> 2)) {
        const int c = cb + (int)(threadIdx.x >> 2);
        double2 *col = A + (size_t)(c < c1 ? c : c0) * lda;
        double2 w = zc(0.0, 0.0);
        if (c < c1)
            for (int i = sub; i < p; i += 4) cfmac(w, x[i], col[i]);
        w.x += __shfl_xor(w.x, 1);
        w.y += __shfl_xor(w.y, 1);
        w.x += __shfl_xor(w.x, 2);
        w.y += __shfl_xor(w.y, 2);
        if (c < c1) {
            w = cadd(w, col[p]);
            const double2 tw = zc(tau * w.x, tau * w.y);
            if (sub == 0) col[p] = csub(col[p], tw);
            for (int i = sub; i < p; i += 4) col[i] = csub(col[i], cmul(x[i], tw));
        }
    }
}

// the current reflector applied to the node's remaining columns 0..jj-1
__global__ void __launch_bounds__(256) k_ubig_left(UlvBig b, int t) {
    const FactArgs &a = b.f;
    const int node = blockIdx.y, m = a.msz[node], r = a.rsz[node], k = m - r;
    const int jj = r - 1 - t;
    const int c0 = blockIdx.x * kUlvChunk;
    if (m == 0 || jj < 0 || c0 >= jj) return;
    const double tau = b.tau[(size_t)node * kUlvMaxM + jj];
    if (tau == 0.0) return;
    double2 *Uw = a.scratch + a.scoff[node];
    const int c1 = c0 + kUlvChunk < jj ? c0 + kUlvChunk : jj;
    ql_apply_cols(Uw + (size_t)jj * m, k + jj, tau, Uw, m, c0, c1);
}

// Q <- H_jj Q, jj = t (Q = H_{r-1} ... H_0)
__global__ void __launch_bounds__(256) k_ubig_q(UlvBig b, int t) {
    const FactArgs &a = b.f;
    const int node = blockIdx.y, m = a.msz[node], r = a.rsz[node], k = m - r;
    const int c0 = blockIdx.x * kUlvChunk;
    if (m == 0 || t >= r || c0 >= m) return;
    const double tau = b.tau[(size_t)node * kUlvMaxM + t];
    if (tau == 0.0) return;
    double2 *Uw = a.scratch + a.scoff[node], *Q = Uw + (size_t)m * m;
    const int c1 = c0 + kUlvChunk < m ? c0 + kUlvChunk : m;
    ql_apply_cols(Uw + (size_t)t * m, k + t, tau, Q, m, c0, c1);
}

__global__ void k_ubig_u2(UlvBig b) {
    const FactArgs &a = b.f;
    const int node = blockIdx.y, m = a.msz[node], r = a.rsz[node], k = m - r;
    if (m == 0) return;
    const double2 *Uw = a.scratch + a.scoff[node];
    double2 *U2 = a.U2 + a.soff[node];
    for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < (long)r * r; e += (long)gridDim.x * blockDim.x) {
        const int i = (int)(e % r), c = (int)(e / r);
        U2[e] = (c <= i) ? Uw[(k + i) + (size_t)c * m] : zc(0.0, 0.0);
    }
}

static int g_ulv_big = 256;        // levels whose largest node has at least this many rows take this path

static void ulv_phase0_big(const FactArgs &fa, int nn, int mlev, int rmax, hipStream_t s) {
    DevBuf tau((size_t)nn * kUlvMaxM * sizeof(double));
    UlvBig b{fa, tau.as<double>()};
    const unsigned y = (unsigned)nn;
    k_ubig_init<<<dim3(256, y), 256, 0, s>>>(b);
    for (int t = 0; t < rmax; ++t) {
        k_ubig_house<<<dim3(1, y), 1024, 0, s>>>(b, t);
        const int ncol = rmax - 1 - t;     // an upper bound of every node's remaining columns
        if (ncol > 0) k_ubig_left<<<dim3((unsigned)((ncol + kUlvChunk - 1) / kUlvChunk), y), kUlvThreads, 0, s>>>(b, t);
    }
    for (int t = 0; t < rmax; ++t)
        k_ubig_q<<<dim3((unsigned)((mlev + kUlvChunk - 1) / kUlvChunk), y), kUlvThreads, 0, s>>>(b, t);
    k_ubig_u2<<<dim3(64, y), 256, 0, s>>>(b);
    FIO_HIP(hipGetLastError());
    FIO_HIP(hipStreamSynchronize(s));   // the reflector scalars are released here
}

// Merge of eq. ulv_merge for every parent (one workgroup per parent):
//   D+ = [[D22(a1), (U2(a2) B U2(a1)^*)^*], [U2(a2) B U2(a1)^*, D22(a2)]],
//   U+ = diag(U2(a1), U2(a2)) U_parent  (skipped at the root).
struct MergeArgs {
    const double2 *D22, *U2;
    const size_t *soff;      // child slots
    const int *rch;          // child ranks
    const double2 *B;        // B_{a2,a1} of each parent
    const size_t *boff;
    const double2 *Upar;     // parent bases (m x r_par slots), or null at the root
    const size_t *upoff;
    const int *rpar;
    double2 *Dout;           // merged D (m x m per parent)
    const size_t *dooff;
    double2 *Uout;           // merged U (m x r_par per parent)
    const size_t *uooff;
    double2 *tmp;            // per parent: T (r2 x r1), then U2(a1)^* (r1 x r1)
    const size_t *toff;
};

// Merge, around four batched GEMMs over the parents of the level:
//   k_ulv_merge_prep: diagonal blocks D22(a1), D22(a2) into D+, and U2(a1)^* next to T;
//   GEMMs: T = U2(a2) B, lower-left block of D+ = T U2(a1)^*, U+ = diag(U2(a1), U2(a2)) U_parent;
//   k_ulv_merge_fill: upper-right block of D+ = conj transpose of the lower-left block.
__global__ void __launch_bounds__(1024) k_ulv_merge_prep(MergeArgs a) {
    const int par = blockIdx.x, tid = threadIdx.x, nt = blockDim.x;
    const int c1 = 2 * par, c2 = 2 * par + 1;
    const int r1 = a.rch[c1], r2 = a.rch[c2], m = r1 + r2;
    if (m == 0) return;
    const double2 *Da = a.D22 + a.soff[c1], *Db = a.D22 + a.soff[c2];
    const double2 *Ua = a.U2 + a.soff[c1];
    double2 *UaH = a.tmp + a.toff[par] + (size_t)r1 * r2;
    double2 *D = a.Dout + a.dooff[par];
    for (int e = tid; e < r1 * r1; e += nt) {
        const int i = e % r1, j = e / r1;
        D[i + (size_t)j * m] = Da[e];
        const double2 u = Ua[j + (size_t)i * r1];
        UaH[e] = zc(u.x, -u.y);
    }
    for (int e = tid; e < r2 * r2; e += nt) {
        const int i = e % r2, j = e / r2;
        D[(r1 + i) + (size_t)(r1 + j) * m] = Db[e];
    }
}

__global__ void __launch_bounds__(1024) k_ulv_merge_fill(MergeArgs a) {
    const int par = blockIdx.x, tid = threadIdx.x, nt = blockDim.x;
    const int r1 = a.rch[2 * par], r2 = a.rch[2 * par + 1], m = r1 + r2;
    double2 *D = a.Dout + a.dooff[par];
    for (int e = tid; e < r1 * r2; e += nt) {
        const int i = e % r1, j = e / r1;          // upper-right (i, r1 + j) = conj(lower-left (r1 + j, i))
        const double2 v = D[(r1 + j) + (size_t)i * m];
        D[i + (size_t)(r1 + j) * m] = zc(v.x, -v.y);
    }
}

// Root: Cholesky of D+ and the explicit inverse Linv of the lower factor, blocked by
// kRootBlock columns: the diagonal blocks and the triangular solves run in small kernels,
// the trailing updates of the Cholesky and of the inverse as GEMMs over the whole GPU.
constexpr int kRootBlock = 64;

__global__ void __launch_bounds__(256) k_root_diag(double2 *D, int m, int k0, int kb, int *fail) {
    __shared__ double sh[16];
    __shared__ int s_flag;
    if (!wg_potrf(D + k0 + (size_t)k0 * m, m, kb, sh, &s_flag))
        if (threadIdx.x == 0) atomicAdd(fail, 1);
}

// rows i >= k0 + kb of the block column: x L_kk^* = a (forward over the kb columns)
__global__ void k_root_panel(double2 *D, int m, int k0, int kb) {
    const int i = k0 + kb + blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= m) return;
    for (int j = 0; j < kb; ++j) {
        double2 acc = D[i + (size_t)(k0 + j) * m];
        for (int l = 0; l < j; ++l) {
            const double2 x = D[i + (size_t)(k0 + l) * m], Ljl = D[(k0 + j) + (size_t)(k0 + l) * m];
            acc.x -= x.x * Ljl.x + x.y * Ljl.y;       // acc -= x conj(Ljl)
            acc.y -= x.y * Ljl.x - x.x * Ljl.y;
        }
        const double d = D[(k0 + j) + (size_t)(k0 + j) * m].x;
        D[i + (size_t)(k0 + j) * m] = zc(acc.x / d, acc.y / d);
    }
}

// PH (kb x rest) = panel^* of D rows k0+kb.., columns k0..k0+kb
__global__ void k_root_ct(const double2 *D, int m, int k0, int kb, double2 *PH) {
    const int rest = m - k0 - kb;
    for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < (long)rest * kb; e += (long)gridDim.x * blockDim.x) {
        const int j = (int)(e % kb), i = (int)(e / kb);
        const double2 v = D[(k0 + kb + i) + (size_t)(k0 + j) * m];
        PH[j + (size_t)i * kb] = zc(v.x, -v.y);
    }
}

__global__ void k_root_clear_upper_and_eye(double2 *D, double2 *X, int m) {
    for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < (long)m * m; e += (long)gridDim.x * blockDim.x) {
        const int i = (int)(e % m), j = (int)(e / m);
        if (j > i) D[e] = zc(0.0, 0.0);
        X[e] = zc(i == j ? 1.0 : 0.0, 0.0);
    }
}

// rows k0..k0+kb of X <- L_kk^{-1} rows k0..k0+kb of X, one lane per column
__global__ void k_root_fwd(const double2 *D, double2 *X, int m, int k0, int kb) {
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= m) return;
    for (int j = 0; j < kb; ++j) {
        double2 acc = X[(k0 + j) + (size_t)c * m];
        for (int l = 0; l < j; ++l) acc = csub(acc, cmul(D[(k0 + j) + (size_t)(k0 + l) * m], X[(k0 + l) + (size_t)c * m]));
        const double d = D[(k0 + j) + (size_t)(k0 + j) * m].x;
        X[(k0 + j) + (size_t)c * m] = zc(acc.x / d, acc.y / d);
    }
}

static void ulv_root_factor(double2 *D, int m, double2 *Linv, int *fail, hipStream_t s) {
    const int nb = kRootBlock;
    DevBuf ph((size_t)nb * m * sizeof(double2) + 16);
    for (int k0 = 0; k0 < m; k0 += nb) {
        const int kb = m - k0 < nb ? m - k0 : nb, rest = m - k0 - kb;
        k_root_diag<<<1, 256, 0, s>>>(D, m, k0, kb, fail);
        if (rest == 0) break;
        k_root_panel<<<(rest + 255) / 256, 256, 0, s>>>(D, m, k0, kb);
        k_root_ct<<<64, 256, 0, s>>>(D, m, k0, kb, ph.as<double2>());
        // trailing update D22 -= P P^* (the whole square; only the lower triangle is used)
        ZgemmDesc d{D + (k0 + kb) + (size_t)k0 * m, ph.as<double2>(), D + (k0 + kb) + (size_t)(k0 + kb) * m,
                    rest, rest, kb, m, kb, m};
        zgemm_one(d, false, zc(-1.0, 0.0), zc(1.0, 0.0), s);
    }
    k_root_clear_upper_and_eye<<<256, 256, 0, s>>>(D, Linv, m);
    // Linv: blocked forward substitution of L X = I
    for (int k0 = 0; k0 < m; k0 += nb) {
        const int kb = m - k0 < nb ? m - k0 : nb, rest = m - k0 - kb;
        k_root_fwd<<<(m + 255) / 256, 256, 0, s>>>(D, Linv, m, k0, kb);
        if (rest == 0) break;
        ZgemmDesc d{D + (k0 + kb) + (size_t)k0 * m, Linv + k0, Linv + (k0 + kb), rest, m, kb, m, m, m};
        zgemm_one(d, false, zc(-1.0, 0.0), zc(1.0, 0.0), s);
    }
    FIO_HIP(hipGetLastError());
    FIO_HIP(hipStreamSynchronize(s));     // the panel buffer is released here
}

// One level of the ULV solve.  UP: z = W y_tau, rows < k to Bh, rows >= k to the parent's
// vector (Ylo).  DOWN: c_tau = W^* [Bh rows; Ylo rows].  32 x 32 output tiles, K through LDS.
struct LevelArgs {
    const double2 *W;
    const size_t *woff;
    const int *m, *k;
    const long *yoff, *roff;
};

// The solve's output: written, or added to what the output holds (accum != 0: the update
// f += G~^{-1} y of a refinement step, fused into the last level)
__device__ __forceinline__ void ulv_store(double2 *p, double2 v, int accum) {
    if (accum) {
        const double2 o = *p;
        v = zc(o.x + v.x, o.y + v.y);
    }
    *p = v;
}

template <bool DOWN>
__global__ void __launch_bounds__(256) k_ulv_level(LevelArgs a, const double2 *__restrict__ Yin, long ldin,
                                                   double2 *__restrict__ Bh, long ldb, double2 *__restrict__ Ylo,
                                                   long ldlo, double2 *__restrict__ Yout, long ldout, int nrhs,
                                                   int tilesN, int accum) {
    const int node = blockIdx.y;
    const int m = a.m[node], k = a.k[node];
    const int tm = blockIdx.x / tilesN, tn = blockIdx.x % tilesN;
    const int m0 = tm * 32, n0 = tn * 32;
    if (m0 >= m || n0 >= nrhs) return;
    const double2 *W = a.W + a.woff[node];
    const long yo = a.yoff[node], ro = a.roff[node];
    __shared__ double2 As[16][33];
    __shared__ double2 Bs[16][33];
    const int tid = threadIdx.x, tx = tid % 16, ty = tid / 16;
    double2 acc[2][2];
#pragma unroll
    for (int x = 0; x < 2; ++x)
#pragma unroll
        for (int y = 0; y < 2; ++y) acc[x][y] = zc(0.0, 0.0);
    for (int k0 = 0; k0 < m; k0 += 16) {
        // all four loads of a thread are issued before any is used (no load inside a thread
        // condition: a thread outside the node or the column block reads W[0] and keeps zero)
        double2 ta[2], tb[2];
        int am[2], ak[2], bk[2], bn[2];
        bool aok[2], bok[2];
#pragma unroll
        for (int q = 0; q < 2; ++q) {
            const int e = tid + 256 * q;
            if (DOWN) {      // op(A) = W^*: element (row, kk) = conj(W(kk, row))
                ak[q] = e % 16;
                am[q] = e / 16;
            } else {
                am[q] = e % 32;
                ak[q] = e / 32;
            }
            const int gm = m0 + am[q], gk = k0 + ak[q];
            aok[q] = gm < m && gk < m;
            ta[q] = W[aok[q] ? (DOWN ? gk + (size_t)gm * m : gm + (size_t)gk * m) : 0];
            bk[q] = e % 16;
            bn[q] = e / 16;
            const int hk = k0 + bk[q], hn = n0 + bn[q];
            bok[q] = hk < m && hn < nrhs;
            const double2 *src;
            if (DOWN)
                src = !bok[q] ? W : (hk < k ? Bh + (yo + hk) + (size_t)hn * ldb : Ylo + (ro + hk - k) + (size_t)hn * ldlo);
            else
                src = !bok[q] ? W : Yin + (yo + hk) + (size_t)hn * ldin;
            tb[q] = *src;
        }
#pragma unroll
        for (int q = 0; q < 2; ++q) {
            const double2 t = DOWN ? zc(ta[q].x, -ta[q].y) : ta[q];
            As[ak[q]][am[q]] = aok[q] ? t : zc(0.0, 0.0);
            Bs[bk[q]][bn[q]] = bok[q] ? tb[q] : zc(0.0, 0.0);
        }
        __syncthreads();
#pragma unroll
        for (int kk = 0; kk < 16; ++kk) {
            double2 a0 = As[kk][tx], a1 = As[kk][tx + 16];
            double2 b0 = Bs[kk][ty], b1 = Bs[kk][ty + 16];
            cfma(acc[0][0], a0, b0);
            cfma(acc[0][1], a0, b1);
            cfma(acc[1][0], a1, b0);
            cfma(acc[1][1], a1, b1);
        }
        __syncthreads();
    }
#pragma unroll
    for (int x = 0; x < 2; ++x) {
        int gm = m0 + tx + 16 * x;
        if (gm >= m) continue;
#pragma unroll
        for (int y = 0; y < 2; ++y) {
            int gn = n0 + ty + 16 * y;
            if (gn >= nrhs) continue;
            if (DOWN)
                ulv_store(Yout + (yo + gm) + (size_t)gn * ldout, acc[x][y], accum);
            else if (gm < k)
                Bh[(yo + gm) + (size_t)gn * ldb] = acc[x][y];
            else
                Ylo[(ro + gm - k) + (size_t)gn * ldlo] = acc[x][y];
        }
    }
}

// The same level product for nodes of at most 64 rows (the leaf level): one workgroup per
// node and 64 right-hand sides, 4 x 4 outputs per thread, so W and the vector block are read
// once and every LDS operand read feeds four multiply-adds; the next 16-deep tiles of both
// operands are fetched into registers while the current ones are used.  Accumulation runs
// over k in the order of k_ulv_level, so both kernels give identical results.
template <bool DOWN>
__global__ void __launch_bounds__(256) k_ulv_level64(LevelArgs a, const double2 *__restrict__ Yin, long ldin,
                                                     double2 *__restrict__ Bh, long ldb, double2 *__restrict__ Ylo,
                                                     long ldlo, double2 *__restrict__ Yout, long ldout, int nrhs,
                                                     int accum) {
    const int node = blockIdx.y;
    const int m = a.m[node], k = a.k[node];
    const int n0 = blockIdx.x * 64;
    if (m == 0 || n0 >= nrhs) return;
    const double2 *W = a.W + a.woff[node];
    const long yo = a.yoff[node], ro = a.roff[node];
    __shared__ double2 As[16][65];
    __shared__ double2 Bs[16][65];
    const int tid = threadIdx.x, tx = tid % 16, ty = tid / 16;
    double2 acc[4][4];
#pragma unroll
    for (int x = 0; x < 4; ++x)
#pragma unroll
        for (int y = 0; y < 4; ++y) acc[x][y] = zc(0.0, 0.0);
    // element r of this thread's share of a 16-deep A / B tile, and its LDS slot
    int amm[4], akk[4], bkk[4], bnn[4];
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const int e = tid + 256 * r;
        if (DOWN) {
            akk[r] = e % 16;
            amm[r] = e / 16;
        } else {
            amm[r] = e % 64;
            akk[r] = e / 64;
        }
        bkk[r] = e % 16;
        bnn[r] = e / 16;
    }
    double2 pa[4], pb[4];
    // The loads carry no branch: a thread outside the node or the column block reads W[0] (the
    // node has m >= 1 rows), and the zeroing and the conjugation of the W^* operand happen when
    // the tile is written to LDS.  With the load inside a thread condition and the conjugation
    // next to it, the compiler waited for each load before issuing the next.
    auto a_ok = [&](int k0, int r) { return amm[r] < m && k0 + akk[r] < m; };
    auto b_ok = [&](int k0, int r) { return k0 + bkk[r] < m && n0 + bnn[r] < nrhs; };
    auto fetch = [&](int k0) {
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int gm = amm[r], gk = k0 + akk[r];
            pa[r] = W[a_ok(k0, r) ? (DOWN ? gk + (size_t)gm * m : gm + (size_t)gk * m) : 0];
        }
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int gk = k0 + bkk[r], gn = n0 + bnn[r];
            const double2 *src;
            if (DOWN)
                src = !b_ok(k0, r) ? W
                                   : (gk < k ? Bh + (yo + gk) + (size_t)gn * ldb : Ylo + (ro + gk - k) + (size_t)gn * ldlo);
            else
                src = !b_ok(k0, r) ? W : Yin + (yo + gk) + (size_t)gn * ldin;
            pb[r] = *src;
        }
    };
    fetch(0);
    for (int k0 = 0; k0 < m; k0 += 16) {
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const double2 t = DOWN ? zc(pa[r].x, -pa[r].y) : pa[r];
            As[akk[r]][amm[r]] = a_ok(k0, r) ? t : zc(0.0, 0.0);
            Bs[bkk[r]][bnn[r]] = b_ok(k0, r) ? pb[r] : zc(0.0, 0.0);
        }
        __syncthreads();
        // the next tile is fetched while this one is used
        if (k0 + 16 < m) fetch(k0 + 16);
#pragma unroll
        for (int kk = 0; kk < 16; ++kk) {
            double2 av[4], bv[4];
#pragma unroll
            for (int x = 0; x < 4; ++x) av[x] = As[kk][tx + 16 * x];
#pragma unroll
            for (int y = 0; y < 4; ++y) bv[y] = Bs[kk][ty + 16 * y];
#pragma unroll
            for (int x = 0; x < 4; ++x)
#pragma unroll
                for (int y = 0; y < 4; ++y) cfma(acc[x][y], av[x], bv[y]);
        }
        __syncthreads();
    }
#pragma unroll
    for (int x = 0; x < 4; ++x) {
        const int gm = tx + 16 * x;
        if (gm >= m) continue;
#pragma unroll
        for (int y = 0; y < 4; ++y) {
            const int gn = n0 + ty + 16 * y;
            if (gn >= nrhs) continue;
            if (DOWN)
                ulv_store(Yout + (yo + gm) + (size_t)gn * ldout, acc[x][y], accum);
            else if (gm < k)
                Bh[(yo + gm) + (size_t)gn * ldb] = acc[x][y];
            else
                Ylo[(ro + gm - k) + (size_t)gn * ldlo] = acc[x][y];
        }
    }
}

// One level of the ULV solve for few right-hand sides on large nodes, in two launches:
// k_ulv_narrow computes partial products over S slices of the inner dimension, one wave
// per 64 output rows and slice, lanes on rows, so W (UP) or W^* (DOWN, the stored copy WH)
// streams coalesced from HBM once; 64-entry pieces of the input vector are staged in LDS
// and read back as broadcasts.  k_ulv_narrow_sum adds the S partials in a fixed order and
// scatters the rows like k_ulv_level.  Partial (s, level row, column) at
// P[(s * rows + row) * 8 + column] for one chunk of 8 columns.
constexpr int kNarrowCols = 8;

template <bool DOWN>
__global__ void __launch_bounds__(64) k_ulv_narrow(LevelArgs a, const double2 *__restrict__ WH,
                                                   const double2 *__restrict__ Yin, long ldin,
                                                   const double2 *__restrict__ Bh, long ldb,
                                                   const double2 *__restrict__ Ylo, long ldlo, int nrhs, int c0,
                                                   int S, long rows, double2 *__restrict__ P) {
    __shared__ double2 xs[64][kNarrowCols];
    const int node = blockIdx.y, sl = blockIdx.z;
    const int m = a.m[node], k = a.k[node];
    const int r0 = blockIdx.x * 64;
    if (r0 >= m) return;
    const int r = r0 + threadIdx.x;
    const int nc = nrhs - c0 < kNarrowCols ? nrhs - c0 : kNarrowCols;
    const double2 *Wn = (DOWN ? WH : a.W) + a.woff[node];
    const long yo = a.yoff[node], ro = a.roff[node];
    const int len = (m + S - 1) / S;
    const int l0 = sl * len, l1 = l0 + len < m ? l0 + len : m;
    double2 acc[kNarrowCols];
#pragma unroll
    for (int c = 0; c < kNarrowCols; ++c) acc[c] = zc(0.0, 0.0);
    for (int lb = l0; lb < l1; lb += 64) {
        const int nl = l1 - lb < 64 ? l1 - lb : 64;
        __syncthreads();
        {
            const int l = lb + threadIdx.x;
            for (int c = 0; c < kNarrowCols; ++c) {
                double2 v = zc(0.0, 0.0);
                if ((int)threadIdx.x < nl && c < nc) {
                    if (DOWN)
                        v = l < k ? Bh[(yo + l) + (size_t)(c0 + c) * ldb] : Ylo[(ro + l - k) + (size_t)(c0 + c) * ldlo];
                    else
                        v = Yin[(yo + l) + (size_t)(c0 + c) * ldin];
                }
                xs[threadIdx.x][c] = v;
            }
        }
        __syncthreads();
        if (r < m) {
            for (int j = 0; j < nl; ++j) {
                const double2 w = Wn[r + (size_t)(lb + j) * m];
#pragma unroll
                for (int c = 0; c < kNarrowCols; ++c) cfma(acc[c], w, xs[j][c]);
            }
        }
    }
    if (r < m) {
        double2 *pp = P + ((size_t)sl * rows + yo + r) * kNarrowCols;
#pragma unroll
        for (int c = 0; c < kNarrowCols; ++c) pp[c] = acc[c];
    }
}

template <bool DOWN>
__global__ void k_ulv_narrow_sum(LevelArgs a, const double2 *__restrict__ P, int S, long rows, int nrhs, int c0,
                                 double2 *__restrict__ Bh, long ldb, double2 *__restrict__ Ylo, long ldlo,
                                 double2 *__restrict__ Yout, long ldout, int accum) {
    const int node = blockIdx.y;
    const int m = a.m[node], k = a.k[node];
    const long yo = a.yoff[node], ro = a.roff[node];
    const int nc = nrhs - c0 < kNarrowCols ? nrhs - c0 : kNarrowCols;
    for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < m * kNarrowCols; e += gridDim.x * blockDim.x) {
        const int r = e / kNarrowCols, c = e % kNarrowCols;
        if (c >= nc) continue;
        double2 v = zc(0.0, 0.0);
        for (int q = 0; q < S; ++q) v = cadd(v, P[((size_t)q * rows + yo + r) * kNarrowCols + c]);
        if (DOWN)
            ulv_store(Yout + (yo + r) + (size_t)(c0 + c) * ldout, v, accum);
        else if (r < k)
            Bh[(yo + r) + (size_t)(c0 + c) * ldb] = v;
        else
            Ylo[(ro + r - k) + (size_t)(c0 + c) * ldlo] = v;
    }
}

// WH = W^* for every node of a level
__global__ void k_ulv_wh(const double2 *W, double2 *WH, const size_t *woff, const int *msz) {
    const int node = blockIdx.y, m = msz[node];
    const double2 *Wn = W + woff[node];
    double2 *Hn = WH + woff[node];
    for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < (long)m * m; e += (long)gridDim.x * blockDim.x) {
        const int i = (int)(e % m), j = (int)(e / m);
        const double2 v = Wn[j + (size_t)i * m];
        Hn[e] = zc(v.x, -v.y);
    }
}

// levels whose largest node has at least this many rows use k_ulv_narrow for <= 16 columns
constexpr int kNarrowMinRows = 128, kNarrowMaxCols = 16;

// inner-dimension slices of a level: about 2048 waves in flight, at least 64 entries per slice,
// and at most 4 N partial rows
static int narrow_slices(long rows, int mmax) {
    const long waves = (rows + 63) / 64;
    long S = (2048 + waves - 1) / waves;
    if (S > mmax / 64) S = mmax / 64;
    if (S > 32) S = 32;
    return S < 1 ? 1 : (int)S;
}

static size_t narrow_part_rows(const hss_ulv_s *f) {
    size_t mx = 0;
    for (int l = 1; l <= f->Lh; ++l) {
        int mm = 0;
        for (int v : f->m[l]) mm = v > mm ? v : mm;
        const size_t need = (size_t)narrow_slices(f->rows[l], mm) * f->rows[l];
        mx = need > mx ? need : mx;
    }
    return mx;
}

template <typename T> static size_t put(std::vector<char> &blob, const std::vector<T> &v) {
    size_t off = (blob.size() + 255) & ~(size_t)255;
    blob.resize(off + v.size() * sizeof(T) + 8);
    if (!v.empty()) std::memcpy(blob.data() + off, v.data(), v.size() * sizeof(T));
    return off;
}

static fio_status factor_impl(hss_s *h, hipStream_t s, hss_ulv_t *out) {
    hss_ulv_s *f = new hss_ulv_s();
    const int Lh = h->Lh;
    f->N = h->N;
    f->leaf = h->leaf;
    f->Lh = Lh;
    f->m.assign(Lh + 1, {});
    f->k.assign(Lh + 1, {});
    f->r.assign(Lh + 1, {});
    f->woff.assign(Lh + 1, {});
    f->yoff.assign(Lh + 1, {});
    f->roff.assign(Lh + 1, {});
    f->rows.assign(Lh + 1, 0);
    fio_status st = guarded([&] {
        size_t wtot = 0;
        for (int l = Lh; l >= 1; --l) {
            const int nn = h->nodes(l);
            long yo = 0, ro = 0;
            for (int j = 0; j < nn; ++j) {
                int m = h->m[l][j], r = h->rank[l][j];
                f->m[l].push_back(m);
                f->r[l].push_back(r);
                f->k[l].push_back(m - r);
                f->woff[l].push_back(wtot);
                wtot += (size_t)m * m;
                f->yoff[l].push_back(yo);
                f->roff[l].push_back(ro);
                yo += m;
                ro += r;
            }
            f->rows[l] = yo;
            f->rows[l - 1] = ro;
        }
        f->m0 = h->m[0][0];
        f->W.alloc(wtot * sizeof(double2) + 16);
        f->Linv.alloc((size_t)f->m0 * f->m0 * sizeof(double2) + 16);
        DevBuf failb(sizeof(int));
        FIO_HIP(hipMemsetAsync(failb.p, 0, sizeof(int), s));
        // level-by-level factorization
        DevBuf Dcur, Ucur, D22, U2, scr, tmp;
        const double2 *Din = h->Dbuf.as<double2>();
        std::vector<size_t> din_off(h->nodes(Lh)), uin_off = h->uoff[Lh];
        for (int j = 0; j < h->nodes(Lh); ++j) din_off[j] = (size_t)j * h->leaf * h->leaf;
        const double2 *Uin = h->Ubuf[Lh]->as<double2>();
        for (int l = Lh; l >= 1; --l) {
            const int nn = h->nodes(l);
            std::vector<size_t> soff(nn), scoff(nn);
            size_t stot = 0, sctot = 0;
            int mlev = 0;
            for (int j = 0; j < nn; ++j) {
                int m = f->m[l][j];
                mlev = m > mlev ? m : mlev;
                soff[j] = stot;
                stot += (size_t)m * m;
                scoff[j] = sctot;
                sctot += (size_t)3 * m * m;
                if (m > kUlvMaxM) throw Err{FIO_ERR_UNSUPPORTED};
            }
            D22.alloc(stot * sizeof(double2) + 16);
            U2.alloc(stot * sizeof(double2) + 16);
            scr.alloc(sctot * sizeof(double2) + 16);
            std::vector<char> blob;
            size_t o_doff = put(blob, din_off), o_uoff = put(blob, uin_off), o_m = put(blob, f->m[l]),
                   o_r = put(blob, f->r[l]), o_w = put(blob, f->woff[l]), o_s = put(blob, soff),
                   o_sc = put(blob, scoff);
            DevBuf meta(blob.size());
            FIO_HIP(hipMemcpyAsync(meta.p, blob.data(), blob.size(), hipMemcpyHostToDevice, s));
            char *mb = meta.as<char>();
            FactArgs fa;
            fa.D = Din;
            fa.doff = (const size_t *)(mb + o_doff);
            fa.U = Uin;
            fa.uoff = (const size_t *)(mb + o_uoff);
            fa.msz = (const int *)(mb + o_m);
            fa.rsz = (const int *)(mb + o_r);
            fa.W = f->W.as<double2>();
            fa.woff = (const size_t *)(mb + o_w);
            fa.D22 = D22.as<double2>();
            fa.U2 = U2.as<double2>();
            fa.soff = (const size_t *)(mb + o_s);
            fa.scratch = scr.as<double2>();
            fa.scoff = (const size_t *)(mb + o_sc);
            fa.fail = failb.as<int>();
            if (mlev < g_ulv_big) {
                k_ulv_node<0><<<nn, ulv_threads(mlev), 0, s>>>(fa);
                FIO_HIP(hipGetLastError());
            } else {
                int rmax = 0;
                for (int v : f->r[l]) rmax = v > rmax ? v : rmax;
                ulv_phase0_big(fa, nn, mlev, rmax, s);
            }
            {
                // Dchk = Q^* D Q for every node of the level: W slot <- Q^* D, T <- (Q^* D) Q
                ZgemmBatch g1, g2;
                double2 *sc = scr.as<double2>();
                double2 *W = f->W.as<double2>();
                for (int j = 0; j < nn; ++j) {
                    const int m = f->m[l][j];
                    double2 *Q = sc + scoff[j] + (size_t)m * m, *T = Q + (size_t)m * m;
                    g1.add(Q, m, Din + din_off[j], m, W + f->woff[l][j], m, m, m, m);
                    g2.add(W + f->woff[l][j], m, Q, m, T, m, m, m, m);
                }
                g1.upload(s);
                g2.upload(s);
                g1.run(true, zc(1.0, 0.0), zc(0.0, 0.0), s);
                g2.run(false, zc(1.0, 0.0), zc(0.0, 0.0), s);
                FIO_HIP(hipStreamSynchronize(s));   // the descriptor lists are released here
            }
            k_ulv_node<1><<<nn, ulv_threads(mlev), 0, s>>>(fa);
            FIO_HIP(hipGetLastError());
            {
                // Dhat22 = Dchk22 - X^* X and W2 = Q2^* - X^* W1 for every node of the level, with
                // X = Dhat21^* (k x r) left in T(0..k, k..m) by the node kernel
                ZgemmBatch g3, g4;
                double2 *sc = scr.as<double2>();
                double2 *W = f->W.as<double2>();
                double2 *D22b = fa.D22;
                for (int j = 0; j < nn; ++j) {
                    const int m = f->m[l][j], r = f->r[l][j], k = m - r;
                    if (m == 0 || r == 0 || k == 0) continue;
                    double2 *T = sc + scoff[j] + 2 * (size_t)m * m;
                    const double2 *X = T + (size_t)k * m;
                    g3.add(X, m, X, m, D22b + soff[j], r, r, r, k);
                    g4.add(X, m, W + f->woff[l][j], m, W + f->woff[l][j] + k, m, r, m, k);
                }
                g3.upload(s);
                g4.upload(s);
                g3.run(true, zc(-1.0, 0.0), zc(1.0, 0.0), s);
                g4.run(true, zc(-1.0, 0.0), zc(1.0, 0.0), s);
                FIO_HIP(hipStreamSynchronize(s));   // the descriptor lists are released here
            }
            // merge into level l-1
            const int np = h->nodes(l - 1);
            std::vector<size_t> dooff(np), uooff(np), toff(np), upoff(np, 0);
            std::vector<int> rpar(np, 0);
            size_t dt = 0, ut = 0, tt = 0;
            for (int j = 0; j < np; ++j) {
                int r1 = f->r[l][2 * j], r2 = f->r[l][2 * j + 1], m = r1 + r2;
                dooff[j] = dt;
                dt += (size_t)m * m;
                toff[j] = tt;
                tt += (size_t)r1 * r2 + (size_t)r1 * r1;      // T, then U2(a1)^*
                if (l - 1 >= 1) {
                    rpar[j] = h->rank[l - 1][j];
                    upoff[j] = h->uoff[l - 1][j];
                }
                uooff[j] = ut;
                ut += (size_t)m * rpar[j];
            }
            DevBuf Dn(dt * sizeof(double2) + 16), Un(ut * sizeof(double2) + 16);
            tmp.alloc(tt * sizeof(double2) + 16);
            std::vector<char> blob2;
            std::vector<size_t> boff = h->boff[l - 1];
            size_t q_s = put(blob2, soff), q_r = put(blob2, f->r[l]), q_b = put(blob2, boff), q_up = put(blob2, upoff),
                   q_rp = put(blob2, rpar), q_do = put(blob2, dooff), q_uo = put(blob2, uooff), q_t = put(blob2, toff);
            DevBuf meta2(blob2.size());
            FIO_HIP(hipMemcpyAsync(meta2.p, blob2.data(), blob2.size(), hipMemcpyHostToDevice, s));
            char *m2 = meta2.as<char>();
            MergeArgs ma;
            ma.D22 = D22.as<double2>();
            ma.U2 = U2.as<double2>();
            ma.soff = (const size_t *)(m2 + q_s);
            ma.rch = (const int *)(m2 + q_r);
            ma.B = h->Bbuf.as<double2>();
            ma.boff = (const size_t *)(m2 + q_b);
            ma.Upar = (l - 1 >= 1) ? h->Ubuf[l - 1]->as<double2>() : nullptr;
            ma.upoff = (const size_t *)(m2 + q_up);
            ma.rpar = (const int *)(m2 + q_rp);
            ma.Dout = Dn.as<double2>();
            ma.dooff = (const size_t *)(m2 + q_do);
            ma.Uout = Un.as<double2>();
            ma.uooff = (const size_t *)(m2 + q_uo);
            ma.tmp = tmp.as<double2>();
            ma.toff = (const size_t *)(m2 + q_t);
            k_ulv_merge_prep<<<np, ulv_threads(mlev), 0, s>>>(ma);
            FIO_HIP(hipGetLastError());
            {
                ZgemmBatch g1, g2, g3, g4;
                const double2 *U2b = U2.as<double2>();
                for (int j = 0; j < np; ++j) {
                    const int r1 = f->r[l][2 * j], r2 = f->r[l][2 * j + 1], m = r1 + r2, rp = rpar[j];
                    if (m == 0) continue;
                    const double2 *Ua = U2b + soff[2 * j], *Ub = U2b + soff[2 * j + 1];
                    double2 *T = tmp.as<double2>() + toff[j], *UaH = T + (size_t)r1 * r2;
                    double2 *Dp = Dn.as<double2>() + dooff[j];
                    g1.add(Ub, r2, h->Bbuf.as<double2>() + boff[j], r2, T, r2, r2, r1, r2);   // T = U2(a2) B
                    g2.add(T, r2, UaH, r1, Dp + r1, m, r2, r1, r1);                          // lower-left
                    if (l - 1 >= 1) {
                        const double2 *Up = h->Ubuf[l - 1]->as<double2>() + upoff[j];
                        double2 *Uo = Un.as<double2>() + uooff[j];
                        g3.add(Ua, r1, Up, m, Uo, m, r1, rp, r1);                            // rows of a1
                        g4.add(Ub, r2, Up + r1, m, Uo + r1, m, r2, rp, r2);                  // rows of a2
                    }
                }
                for (ZgemmBatch *g : {&g1, &g2, &g3, &g4}) g->upload(s);
                for (ZgemmBatch *g : {&g1, &g2, &g3, &g4}) g->run(false, zc(1.0, 0.0), zc(0.0, 0.0), s);
                k_ulv_merge_fill<<<np, ulv_threads(mlev), 0, s>>>(ma);
                FIO_HIP(hipGetLastError());
                FIO_HIP(hipStreamSynchronize(s));   // the descriptor lists are released here
            }
            int fail = 0;
            FIO_HIP(hipMemcpy(&fail, failb.p, sizeof(int), hipMemcpyDeviceToHost));
            if (fail) throw Err{FIO_ERR_NOT_HPD};
            Dcur.swap(Dn);
            Ucur.swap(Un);
            Din = Dcur.as<double2>();
            Uin = Ucur.as<double2>();
            din_off = dooff;
            uin_off = uooff;
        }
        if (f->m0 > 0) {
            ulv_root_factor(Dcur.as<double2>(), f->m0, f->Linv.as<double2>(), failb.as<int>(), s);
            int fail = 0;
            FIO_HIP(hipMemcpy(&fail, failb.p, sizeof(int), hipMemcpyDeviceToHost));
            if (fail) throw Err{FIO_ERR_NOT_HPD};
        }
        // device tables for the solve
        std::vector<char> blob;
        f->meta_woff.assign(Lh + 1, 0);
        f->meta_m.assign(Lh + 1, 0);
        f->meta_k.assign(Lh + 1, 0);
        f->meta_yoff.assign(Lh + 1, 0);
        f->meta_roff.assign(Lh + 1, 0);
        for (int l = 1; l <= Lh; ++l) {
            f->meta_woff[l] = put(blob, f->woff[l]);
            f->meta_m[l] = put(blob, f->m[l]);
            f->meta_k[l] = put(blob, f->k[l]);
            f->meta_yoff[l] = put(blob, f->yoff[l]);
            f->meta_roff[l] = put(blob, f->roff[l]);
        }
        f->meta.alloc(blob.size() + 16);
        FIO_HIP(hipMemcpy(f->meta.p, blob.data(), blob.size(), hipMemcpyHostToDevice));
        // W^* copies for the levels that the narrow solve kernel serves
        bool any = false;
        for (int l = 1; l <= Lh; ++l)
            for (int v : f->m[l]) any = any || v >= kNarrowMinRows;
        if (any) {
            f->WH.alloc(wtot * sizeof(double2) + 16);
            const char *mb = f->meta.as<char>();
            for (int l = 1; l <= Lh; ++l) {
                int ml = 0;
                for (int v : f->m[l]) ml = v > ml ? v : ml;
                if (ml < kNarrowMinRows) continue;
                k_ulv_wh<<<dim3(64, (unsigned)f->m[l].size()), 256, 0, s>>>(
                    f->W.as<double2>(), f->WH.as<double2>(), (const size_t *)(mb + f->meta_woff[l]),
                    (const int *)(mb + f->meta_m[l]));
            }
            FIO_HIP(hipGetLastError());
            FIO_HIP(hipStreamSynchronize(s));
        }
        return FIO_OK;
    });
    if (st != FIO_OK) {
        delete f;
        return st;
    }
    *out = f;
    return FIO_OK;
}

static size_t ulv_ws_bytes(const hss_ulv_s *f, int nrhs) {
    // level vectors l = 0..Lh-1, Bh for l = 1..Lh, root temporary
    size_t rows = 0;
    for (int l = 0; l < f->Lh; ++l) rows += f->rows[l];
    for (int l = 1; l <= f->Lh; ++l) rows += f->rows[l];
    rows += f->m0;
    size_t part = 0;
    if (f->WH.p && nrhs <= kNarrowMaxCols) part = narrow_part_rows(f) * kNarrowCols;   // entries
    return (rows + 8 * (size_t)(f->Lh + 2)) * (size_t)nrhs * sizeof(double2) + part * sizeof(double2) + 8192;
}

// C = G~^{-1} Y, or C += G~^{-1} Y with accumulate (the last level adds to C)
void ulv_solve_impl(hss_ulv_s *f, const double2 *Y, long ldy, double2 *C, long ldc, int nrhs, void *ws,
                    hipStream_t s, bool accumulate = false) {
    if (nrhs <= 0) return;
    const int Lh = f->Lh;
    double2 *base = reinterpret_cast<double2 *>(ws);
    std::vector<double2 *> Yl(Lh + 1, nullptr), Bl(Lh + 1, nullptr);
    size_t off = 0;
    auto take = [&](long rows) {
        double2 *p = base + off;
        off += ((size_t)rows * nrhs + 7) & ~(size_t)7;
        return p;
    };
    for (int l = 0; l < Lh; ++l) Yl[l] = take(f->rows[l]);
    for (int l = 1; l <= Lh; ++l) Bl[l] = take(f->rows[l]);
    double2 *rt = take(f->m0);
    const char *mb = f->meta.as<char>();
    auto args = [&](int l) {
        LevelArgs a;
        a.W = f->W.as<double2>();
        a.woff = (const size_t *)(mb + f->meta_woff[l]);
        a.m = (const int *)(mb + f->meta_m[l]);
        a.k = (const int *)(mb + f->meta_k[l]);
        a.yoff = (const long *)(mb + f->meta_yoff[l]);
        a.roff = (const long *)(mb + f->meta_roff[l]);
        return a;
    };
    const int tilesN = (nrhs + 31) / 32;
    auto mmax = [&](int l) {
        int v = 0;
        for (int x : f->m[l]) v = x > v ? x : v;
        return v;
    };
    // few right-hand sides on large nodes: rows on lanes, W streamed once per 8 columns
    // (k_ulv_narrow), over S slices of the inner dimension so that about 2048 waves stream
    auto narrow = [&](int l) { return nrhs <= kNarrowMaxCols && f->WH.p && mmax(l) >= kNarrowMinRows; };
    auto slices = [&](int l) { return narrow_slices(f->rows[l], mmax(l)); };
    double2 *part = nullptr;
    if (f->WH.p && nrhs <= kNarrowMaxCols) {
        part = base + off;
        off += narrow_part_rows(f) * kNarrowCols;
    }
    // bottom-up
    for (int l = Lh; l >= 1; --l) {
        const int tilesM = (mmax(l) + 31) / 32;
        if (tilesM == 0) continue;
        const double2 *yin = (l == Lh) ? Y : Yl[l];
        long ldin = (l == Lh) ? ldy : f->rows[l];
        FIO_TIMED("ulv_up", s);
        if (narrow(l)) {
            const int S = slices(l);
            for (int c0 = 0; c0 < nrhs; c0 += kNarrowCols) {
                dim3 g((unsigned)((mmax(l) + 63) / 64), (unsigned)f->m[l].size(), (unsigned)S);
                k_ulv_narrow<false><<<g, 64, 0, s>>>(args(l), nullptr, yin, ldin, nullptr, 0, nullptr, 0, nrhs, c0,
                                                     S, f->rows[l], part);
                dim3 g2((unsigned)((mmax(l) * kNarrowCols + 255) / 256), (unsigned)f->m[l].size());
                k_ulv_narrow_sum<false><<<g2, 256, 0, s>>>(args(l), part, S, f->rows[l], nrhs, c0, Bl[l], f->rows[l],
                                                           Yl[l - 1], f->rows[l - 1], nullptr, 0, 0);
            }
        } else if (mmax(l) > 32 && mmax(l) <= 64) {
            dim3 grid((unsigned)((nrhs + 63) / 64), f->m[l].size());
            k_ulv_level64<false><<<grid, 256, 0, s>>>(args(l), yin, ldin, Bl[l], f->rows[l], Yl[l - 1],
                                                      f->rows[l - 1], nullptr, 0, nrhs, 0);
        } else {
            dim3 grid(tilesM * tilesN, f->m[l].size());
            k_ulv_level<false><<<grid, 256, 0, s>>>(args(l), yin, ldin, Bl[l], f->rows[l], Yl[l - 1], f->rows[l - 1],
                                                    nullptr, 0, nrhs, tilesN, 0);
        }
    }
    // root: Y0 <- Linv^* Linv Y0
    if (f->m0 > 0) {
        ZgemmDesc d0{f->Linv.as<double2>(), Yl[0], rt, f->m0, nrhs, f->m0, f->m0, f->m0, f->m0};
        ZgemmDesc d1{f->Linv.as<double2>(), rt, Yl[0], f->m0, nrhs, f->m0, f->m0, f->m0, f->m0};
        FIO_TIMED("ulv_root", s);
        zgemm_one(d0, false, zc(1.0), zc(0.0), s);
        zgemm_one(d1, true, zc(1.0), zc(0.0), s);
    }
    // top-down
    for (int l = 1; l <= Lh; ++l) {
        const int tilesM = (mmax(l) + 31) / 32;
        if (tilesM == 0) continue;
        double2 *yout = (l == Lh) ? C : Yl[l];
        long ldout = (l == Lh) ? ldc : f->rows[l];
        const int acc_l = (l == Lh && accumulate) ? 1 : 0;
        FIO_TIMED("ulv_down", s);
        if (narrow(l)) {
            const int S = slices(l);
            for (int c0 = 0; c0 < nrhs; c0 += kNarrowCols) {
                dim3 g((unsigned)((mmax(l) + 63) / 64), (unsigned)f->m[l].size(), (unsigned)S);
                k_ulv_narrow<true><<<g, 64, 0, s>>>(args(l), f->WH.as<double2>(), nullptr, 0, Bl[l], f->rows[l],
                                                    Yl[l - 1], f->rows[l - 1], nrhs, c0, S, f->rows[l], part);
                dim3 g2((unsigned)((mmax(l) * kNarrowCols + 255) / 256), (unsigned)f->m[l].size());
                k_ulv_narrow_sum<true><<<g2, 256, 0, s>>>(args(l), part, S, f->rows[l], nrhs, c0, nullptr, 0,
                                                          nullptr, 0, yout, ldout, acc_l);
            }
        } else if (mmax(l) > 32 && mmax(l) <= 64) {
            dim3 grid((unsigned)((nrhs + 63) / 64), f->m[l].size());
            k_ulv_level64<true><<<grid, 256, 0, s>>>(args(l), nullptr, 0, Bl[l], f->rows[l], Yl[l - 1],
                                                     f->rows[l - 1], yout, ldout, nrhs, acc_l);
        } else {
            dim3 grid(tilesM * tilesN, f->m[l].size());
            k_ulv_level<true><<<grid, 256, 0, s>>>(args(l), nullptr, 0, Bl[l], f->rows[l], Yl[l - 1], f->rows[l - 1],
                                                   yout, ldout, nrhs, tilesN, acc_l);
        }
    }
    FIO_HIP(hipGetLastError());
}

size_t ulv_ws_bytes_pub(const hss_ulv_s *f, int nrhs) { return ulv_ws_bytes(f, nrhs); }

}  // namespace fio

using namespace fio;

extern "C" fio_status hss_ulv_factor(hss_t h, void *stream, hss_ulv_t *out) {
    FIO_CHECK_ARG(h && out);
    return factor_impl(h, as_stream(stream), out);
}

extern "C" fio_status hss_ulv_workspace_size(hss_ulv_t f, int nrhs, size_t *bytes) {
    FIO_CHECK_ARG(f && bytes && nrhs >= 0);
    *bytes = ulv_ws_bytes(f, nrhs);
    return FIO_OK;
}

extern "C" fio_status hss_ulv_solve(hss_ulv_t f, const void *Y, long ldy, void *C, long ldc, int nrhs, void *ws,
                                    size_t ws_bytes, void *stream) {
    FIO_CHECK_ARG(f && nrhs >= 0);
    if (nrhs == 0) return FIO_OK;
    FIO_CHECK_ARG(Y && C && ldy >= f->N && ldc >= f->N);
    if (Y == C) FIO_CHECK_ARG(ldy == ldc);
    size_t need = ulv_ws_bytes(f, nrhs);
    return guarded([&] {
        hipStream_t s = as_stream(stream);
        if (ws) {
            if (ws_bytes < need) return FIO_ERR_ARG;
            ulv_solve_impl(f, (const double2 *)Y, ldy, (double2 *)C, ldc, nrhs, ws, s);
        } else {
            std::lock_guard<std::mutex> lk(f->ws_mu);
            if (f->ws.bytes < need) {
                FIO_HIP(hipStreamSynchronize(s));
                f->ws.alloc(need);
            }
            ulv_solve_impl(f, (const double2 *)Y, ldy, (double2 *)C, ldc, nrhs, f->ws.p, s);
        }
        return FIO_OK;
    });
}

extern "C" void hss_ulv_destroy(hss_ulv_t f) { delete f; }

extern "C" void fio_ulv_set_big_node(int rows) { fio::g_ulv_big = rows > 0 ? rows : 256; }
