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

static_assert(kMaxCoarseCols <= kBlock, "the coarse-level kernels hold one column per thread");

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

// out[j] = sum_i A[j][i] v[i] for the K columns of A: one work-group per column, four
// independent partial sums per thread to keep loads in flight.
__global__ void __launch_bounds__(kBlock) k_coarse_dots(const double* __restrict__ A, int N,
                                                        const double* __restrict__ v, double* __restrict__ out) {
    const double* a = A + (size_t)blockIdx.x * N;
    double p[4] = {0.0, 0.0, 0.0, 0.0};
    int i = threadIdx.x;
    for (; i + 3 * kBlock < N; i += 4 * kBlock) {
#pragma unroll
        for (int u = 0; u < 4; ++u) p[u] += a[i + u * kBlock] * v[i + u * kBlock];
    }
    for (; i < N; i += kBlock) p[0] += a[i] * v[i];
    const double s = wg_sum((p[0] + p[1]) + (p[2] + p[3]));
    if (threadIdx.x == 0) out[blockIdx.x] = s;
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

// out = x + Y c with c = base + sgn Einv d (Einv K x K and symmetric, base may be null = 0):
// every work-group forms c in LDS from d (thread j sums column j of Einv, which is row j, so
// the threads' loads are contiguous; the same order in every block), then one thread per
// entry sums its K column values. Block 0 writes Einv d to a_out (may be null).
__global__ void __launch_bounds__(kBlock) k_coarse_update(const double* __restrict__ Einv, const double* __restrict__ d,
                                                          const double* __restrict__ base, int K, double sgn,
                                                          const double* __restrict__ Y, int N,
                                                          const double* __restrict__ x, double* __restrict__ out,
                                                          double* __restrict__ a_out) {
    __shared__ double ds[kMaxCoarseCols];
    __shared__ double c[kMaxCoarseCols];
    __shared__ double part[kBlock];
    for (int j = threadIdx.x; j < K; j += kBlock) ds[j] = d[j];
    __syncthreads();
    // Einv d over all threads: row j split into `parts` chunks of its columns (threads of one
    // chunk read contiguous entries), four independent partial sums per thread
    const int parts = kBlock / K;  // >= 1 (K <= kMaxCoarseCols = kBlock); parts * K <= kBlock
    const int chunk = (K + parts - 1) / parts;
    const int t = threadIdx.x;
    if (t < parts * K) {
        const int j = t % K, l0 = (t / K) * chunk, l1 = l0 + chunk < K ? l0 + chunk : K;
        double p[4] = {0.0, 0.0, 0.0, 0.0};
        int l = l0;
        for (; l + 3 < l1; l += 4) {
#pragma unroll
            for (int u = 0; u < 4; ++u) p[u] += Einv[(size_t)(l + u) * K + j] * ds[l + u];
        }
        for (; l < l1; ++l) p[0] += Einv[(size_t)l * K + j] * ds[l];
        part[t] = (p[0] + p[1]) + (p[2] + p[3]);
    }
    __syncthreads();
    for (int j = threadIdx.x; j < K; j += kBlock) {
        double s = 0.0;
        for (int pi = 0; pi < parts; ++pi) s += part[pi * K + j];
        c[j] = (base ? base[j] : 0.0) + sgn * s;
        if (a_out && blockIdx.x == 0) a_out[j] = s;
    }
    __syncthreads();
    const int i = blockIdx.x * kBlock + threadIdx.x;
    if (i >= N) return;
    double p[4] = {0.0, 0.0, 0.0, 0.0};
    int j = 0;
    for (; j + 3 < K; j += 4) {
#pragma unroll
        for (int u = 0; u < 4; ++u) p[u] += Y[(size_t)(j + u) * N + i] * c[j + u];
    }
    for (; j < K; ++j) p[0] += Y[(size_t)j * N + i] * c[j];
    out[i] = x[i] + ((p[0] + p[1]) + (p[2] + p[3]));
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

void launch_coarse_dots(hipStream_t st, const double* A, int N, int K, const double* v, double* out) {
    hipLaunchKernelGGL(k_coarse_dots, dim3(K), dim3(kBlock), 0, st, A, N, v, out);
}

void launch_coarse_update(hipStream_t st, const double* Einv, const double* d, const double* base, int K, double sgn,
                          const double* Y, int N, const double* x, double* out, double* a_out) {
    if (N <= 0) return;
    hipLaunchKernelGGL(k_coarse_update, dim3(nblocks(N)), dim3(kBlock), 0, st, Einv, d, base, K, sgn, Y, N, x, out,
                       a_out);
}

}  // namespace brd
