// Fourier coarse level of the Schur preconditioner: the basis of low Fourier modes
// of the blob set, its Galerkin matrix E = Z^T (M Z), and the small dense pieces
// of the balancing two-level apply
//   B r = Q r + (I - Q M) W (I - M Q) r,   Q = Z E^{-1} Z^T,
// (Mandel's balancing form) for N-vectors. Columns are stored one after another:
// column j of an N x K block is [j * N, (j + 1) * N). Every reduction runs in a
// fixed order, so results are reproducible.
#include "brd.hpp"
#include "launch.hpp"

namespace brd {

// Column 2t = cos(k_t . q_i), column 2t + 1 = sin(k_t . q_i), with
// k_t = 2 pi (m_x / L_x, m_y / L_y, m_z / L_z) from the integer table mv (3 per mode).
__global__ void k_coarse_basis(const double* __restrict__ q, int N, const int* __restrict__ mv, double kx, double ky,
                               double kz, double* __restrict__ Z) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const int t = blockIdx.y;
    if (i >= N) return;
    const double ph = ((double)mv[3 * t] * kx) * q[3 * i] + ((double)mv[3 * t + 1] * ky) * q[3 * i + 1] +
                      ((double)mv[3 * t + 2] * kz) * q[3 * i + 2];
    double s, c;
    sincos(ph, &s, &c);
    Z[(size_t)(2 * t) * N + i] = c;
    Z[(size_t)(2 * t + 1) * N + i] = s;
}

// One work-group per column: remove the column's mean over the blobs.
__global__ void __launch_bounds__(kBlock) k_coarse_center(double* __restrict__ Z, int N) {
    double* z = Z + (size_t)blockIdx.x * N;
    double s = 0.0;
    for (int i = threadIdx.x; i < N; i += kBlock) s += z[i];
    const double m = wg_sum(s) / (double)N;
    for (int i = threadIdx.x; i < N; i += kBlock) z[i] -= m;
}

// part[j][s] = sum_{i in chunk s} A[j][i] v[i] for the K columns of A and the row chunks
// [s kCoarseChunk, (s + 1) kCoarseChunk): one work-group per (chunk, column) so the grid fills
// the chip, four independent partial sums per thread to keep loads in flight. A grid of K + 1
// columns adds the chunk sums of v itself as column K.
__global__ void __launch_bounds__(kBlock) k_coarse_dots(const double* __restrict__ A, int N, int K,
                                                        const double* __restrict__ v, double* __restrict__ part) {
    const int s = blockIdx.x, j = blockIdx.y;
    if (j == K) {
        const int i1 = min(N, (s + 1) * kCoarseChunk);
        double p[4] = {0.0, 0.0, 0.0, 0.0};
        int i = s * kCoarseChunk + threadIdx.x;
        for (; i + 3 * kBlock < i1; i += 4 * kBlock) {
#pragma unroll
            for (int u = 0; u < 4; ++u) p[u] += v[i + u * kBlock];
        }
        for (; i < i1; i += kBlock) p[0] += v[i];
        const double t = wg_sum((p[0] + p[1]) + (p[2] + p[3]));
        if (threadIdx.x == 0) part[(size_t)j * gridDim.x + s] = t;
        return;
    }
    const double* a = A + (size_t)j * N;
    const int i1 = min(N, (s + 1) * kCoarseChunk);
    double p[4] = {0.0, 0.0, 0.0, 0.0};
    int i = s * kCoarseChunk + threadIdx.x;
    for (; i + 3 * kBlock < i1; i += 4 * kBlock) {
#pragma unroll
        for (int u = 0; u < 4; ++u) p[u] += a[i + u * kBlock] * v[i + u * kBlock];
    }
    for (; i < i1; i += kBlock) p[0] += a[i] * v[i];
    const double t = wg_sum((p[0] + p[1]) + (p[2] + p[3]));
    if (threadIdx.x == 0) part[(size_t)j * gridDim.x + s] = t;
}

// E[a][b] = sum_i Z[a][i] Y[b][i]: one work-group per entry (grid K x K).
__global__ void __launch_bounds__(kBlock) k_coarse_gram(const double* __restrict__ Z, const double* __restrict__ Y,
                                                        int N, int K, double* __restrict__ E) {
    const double* za = Z + (size_t)blockIdx.y * N;
    const double* yb = Y + (size_t)blockIdx.x * N;
    double p[4] = {0.0, 0.0, 0.0, 0.0};
    int i = threadIdx.x;
    for (; i + 3 * kBlock < N; i += 4 * kBlock) {
#pragma unroll
        for (int u = 0; u < 4; ++u) p[u] += za[i + u * kBlock] * yb[i + u * kBlock];
    }
    for (; i < N; i += kBlock) p[0] += za[i] * yb[i];
    const double s = wg_sum((p[0] + p[1]) + (p[2] + p[3]));
    if (threadIdx.x == 0) E[(size_t)blockIdx.y * K + blockIdx.x] = s;
}

// out = (x - xm) + Y c with c = base + sgn d, d[j] = sum_s part[j][s] over the S chunk sums of
// k_coarse_dots (base may be null = 0) and, with sub_mean, xm the mean of x from column K of
// part (0 otherwise). A work-group takes 64 rows: every block forms c and xm in LDS (the same
// order in every block), then wave w sums the rows' values of its quarter of the columns and
// the four quarters are added in a fixed order. Block 0 writes d to a_out (may be null).
__global__ void __launch_bounds__(kBlock) k_coarse_update(const double* __restrict__ part, int S,
                                                          const double* __restrict__ base, int K, double sgn,
                                                          const double* __restrict__ Y, int N,
                                                          const double* __restrict__ x, double* __restrict__ out,
                                                          double* __restrict__ a_out, int sub_mean) {
    __shared__ double c[kMaxCoarseCols + 1];
    __shared__ double q[kBlock];
    const int kc = K + (sub_mean ? 1 : 0);
    for (int j = threadIdx.x; j < kc; j += kBlock) {
        const double* pj = part + (size_t)j * S;
        double t = 0.0;
        for (int s = 0; s < S; ++s) t += pj[s];
        if (j == K) {
            c[j] = t / (double)N;
        } else {
            c[j] = (base ? base[j] : 0.0) + sgn * t;
            if (a_out && blockIdx.x == 0) a_out[j] = t;
        }
    }
    __syncthreads();
    const double xm = sub_mean ? c[K] : 0.0;
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int i = blockIdx.x * 64 + lane;
    const int kq = (K + 3) >> 2;
    const int j0 = w * kq, j1 = min(K, j0 + kq);
    double p[4] = {0.0, 0.0, 0.0, 0.0};
    if (i < N) {
        int j = j0;
        for (; j + 3 < j1; j += 4) {
#pragma unroll
            for (int u = 0; u < 4; ++u) p[u] += Y[(size_t)(j + u) * N + i] * c[j + u];
        }
        for (; j < j1; ++j) p[0] += Y[(size_t)j * N + i] * c[j];
    }
    q[threadIdx.x] = (p[0] + p[1]) + (p[2] + p[3]);
    __syncthreads();
    if (w == 0 && i < N) out[i] = (x[i] - xm) + ((q[lane] + q[64 + lane]) + (q[128 + lane] + q[192 + lane]));
}

// out column j = sum_l Y column l * Einv[l][j]: the basis with E^{-1} folded in, so that the
// apply's coefficients E^{-1} Z^T r are plain dot products (Einv symmetric).
__global__ void __launch_bounds__(kBlock) k_coarse_rotate(const double* __restrict__ Y, const double* __restrict__ Einv,
                                                          int N, int K, double* __restrict__ out) {
    const int i = blockIdx.x * kBlock + threadIdx.x;
    const int j = blockIdx.y;
    if (i >= N) return;
    double p[4] = {0.0, 0.0, 0.0, 0.0};
    int l = 0;
    for (; l + 3 < K; l += 4) {
#pragma unroll
        for (int u = 0; u < 4; ++u) p[u] += Y[(size_t)(l + u) * N + i] * Einv[(size_t)(l + u) * K + j];
    }
    for (; l < K; ++l) p[0] += Y[(size_t)l * N + i] * Einv[(size_t)l * K + j];
    out[(size_t)j * N + i] = (p[0] + p[1]) + (p[2] + p[3]);
}

void launch_coarse_basis(hipStream_t st, const double* q, int N, const int* mv, int nmodes, double kx, double ky,
                         double kz, double* Z) {
    if (N <= 0 || nmodes <= 0) return;
    hipLaunchKernelGGL(k_coarse_basis, dim3(nblocks(N), nmodes), dim3(kBlock), 0, st, q, N, mv, kx, ky, kz, Z);
    hipLaunchKernelGGL(k_coarse_center, dim3(2 * nmodes), dim3(kBlock), 0, st, Z, N);
}

void launch_coarse_gram(hipStream_t st, const double* Z, const double* Y, int N, int K, double* E) {
    hipLaunchKernelGGL(k_coarse_gram, dim3(K, K), dim3(kBlock), 0, st, Z, Y, N, K, E);
}

int coarse_chunks(int N) { return N > 0 ? (N + kCoarseChunk - 1) / kCoarseChunk : 0; }

void launch_coarse_dots(hipStream_t st, const double* A, int N, int K, const double* v, double* part, bool with_sum) {
    if (N <= 0) return;
    hipLaunchKernelGGL(k_coarse_dots, dim3(coarse_chunks(N), K + (with_sum ? 1 : 0)), dim3(kBlock), 0, st, A, N, K, v,
                       part);
}

void launch_coarse_update(hipStream_t st, const double* part, const double* base, int K, double sgn, const double* Y,
                          int N, const double* x, double* out, double* a_out, bool sub_mean) {
    if (N <= 0) return;
    hipLaunchKernelGGL(k_coarse_update, dim3((N + 63) / 64), dim3(kBlock), 0, st, part, coarse_chunks(N), base, K, sgn,
                       Y, N, x, out, a_out, sub_mean ? 1 : 0);
}

void launch_coarse_rotate(hipStream_t st, const double* Y, const double* Einv, int N, int K, double* out) {
    if (N <= 0) return;
    hipLaunchKernelGGL(k_coarse_rotate, dim3(nblocks(N), K), dim3(kBlock), 0, st, Y, Einv, N, K, out);
}

}  // namespace brd
