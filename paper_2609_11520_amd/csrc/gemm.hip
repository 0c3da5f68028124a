// Batched variable-size complex128 GEMM: C_b = alpha op(A_b) B_b + beta C_b.
// One workgroup of 256 threads computes a 32 x 32 tile of one batch entry;
// K is consumed in slices of 16 staged through LDS (coalesced loads along the
// contiguous dimension of each operand).  Used for the HSS basis lifts and
// projections, the ULV solve levels and the telescoping HSS matvec.
#include "common.h"

namespace fio {

constexpr int TM = 32, TN = 32, TK = 16;

template <bool CONJA, bool BETA>
__device__ __forceinline__ void tile_zgemm(const ZgemmDesc &d, int tilesN, double2 alpha, double2 beta) {
    const int tm = blockIdx.x / tilesN, tn = blockIdx.x % tilesN;
    const int m0 = tm * TM, n0 = tn * TN;
    if (m0 >= d.M || n0 >= d.N) return;
    __shared__ double2 As[TK][TM + 1];
    __shared__ double2 Bs[TK][TN + 1];
    const int tid = threadIdx.x;
    const int tx = tid % 16, ty = tid / 16;
    double2 acc[2][2];
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b) acc[a][b] = zc(0.0, 0.0);
    for (int k0 = 0; k0 < d.K; k0 += TK) {
        for (int e = tid; e < TM * TK; e += 256) {
            int mm, kk;
            if (CONJA) {
                kk = e % TK;
                mm = e / TK;
            } else {
                mm = e % TM;
                kk = e / TM;
            }
            int gm = m0 + mm, gk = k0 + kk;
            double2 v = zc(0.0, 0.0);
            if (gm < d.M && gk < d.K) {
                if (CONJA) {
                    double2 t = d.A[gk + (size_t)gm * d.lda];
                    v = zc(t.x, -t.y);
                } else {
                    v = d.A[gm + (size_t)gk * d.lda];
                }
            }
            As[kk][mm] = v;
        }
        for (int e = tid; e < TK * TN; e += 256) {
            int kk = e % TK, nn = e / TK;
            int gk = k0 + kk, gn = n0 + nn;
            Bs[kk][nn] = (gk < d.K && gn < d.N) ? d.B[gk + (size_t)gn * d.ldb] : zc(0.0, 0.0);
        }
        __syncthreads();
#pragma unroll
        for (int kk = 0; kk < TK; ++kk) {
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
    for (int a = 0; a < 2; ++a) {
        int gm = m0 + tx + 16 * a;
        if (gm >= d.M) continue;
#pragma unroll
        for (int b = 0; b < 2; ++b) {
            int gn = n0 + ty + 16 * b;
            if (gn >= d.N) continue;
            double2 *cp = d.C + gm + (size_t)gn * d.ldc;
            double2 r = cmul(alpha, acc[a][b]);
            if (BETA) r = cadd(r, cmul(beta, *cp));
            *cp = r;
        }
    }
}

template <bool CONJA, bool BETA>
__global__ void __launch_bounds__(256) k_zgemm_vb(const ZgemmDesc *__restrict__ descs, int tilesN, double2 alpha,
                                                  double2 beta) {
    tile_zgemm<CONJA, BETA>(descs[blockIdx.y], tilesN, alpha, beta);
}

template <bool CONJA, bool BETA>
__global__ void __launch_bounds__(256) k_zgemm_one(ZgemmDesc d, int tilesN, double2 alpha, double2 beta) {
    tile_zgemm<CONJA, BETA>(d, tilesN, alpha, beta);
}

void zgemm_one(const ZgemmDesc &d, bool conjA, double2 alpha, double2 beta, hipStream_t s) {
    if (d.M <= 0 || d.N <= 0) return;
    int tilesM = (d.M + TM - 1) / TM, tilesN = (d.N + TN - 1) / TN;
    const bool useBeta = !(beta.x == 0.0 && beta.y == 0.0);
    dim3 grid(tilesM * tilesN, 1);
    if (conjA) {
        if (useBeta)
            k_zgemm_one<true, true><<<grid, 256, 0, s>>>(d, tilesN, alpha, beta);
        else
            k_zgemm_one<true, false><<<grid, 256, 0, s>>>(d, tilesN, alpha, beta);
    } else {
        if (useBeta)
            k_zgemm_one<false, true><<<grid, 256, 0, s>>>(d, tilesN, alpha, beta);
        else
            k_zgemm_one<false, false><<<grid, 256, 0, s>>>(d, tilesN, alpha, beta);
    }
    FIO_HIP(hipGetLastError());
}

void zgemm_vbatched(const ZgemmDesc *d_descs, int count, int maxM, int maxN, bool conjA, double2 alpha,
                    double2 beta, hipStream_t s) {
    if (count <= 0 || maxM <= 0 || maxN <= 0) return;
    int tilesM = (maxM + TM - 1) / TM, tilesN = (maxN + TN - 1) / TN;
    const bool useBeta = !(beta.x == 0.0 && beta.y == 0.0);
    // gridDim.y is limited to 65535 entries per launch
    for (int off = 0; off < count; off += 65535) {
        int cnt = count - off < 65535 ? count - off : 65535;
        dim3 grid(tilesM * tilesN, cnt);
        if (conjA) {
            if (useBeta)
                k_zgemm_vb<true, true><<<grid, 256, 0, s>>>(d_descs + off, tilesN, alpha, beta);
            else
                k_zgemm_vb<true, false><<<grid, 256, 0, s>>>(d_descs + off, tilesN, alpha, beta);
        } else {
            if (useBeta)
                k_zgemm_vb<false, true><<<grid, 256, 0, s>>>(d_descs + off, tilesN, alpha, beta);
            else
                k_zgemm_vb<false, false><<<grid, 256, 0, s>>>(d_descs + off, tilesN, alpha, beta);
        }
    }
    FIO_HIP(hipGetLastError());
}

}  // namespace fio
