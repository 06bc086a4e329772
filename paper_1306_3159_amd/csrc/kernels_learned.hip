// Learned pairwise preconditioner for the Schur complement M = J A^+ S.
//
// The paper's diagonal preconditioner M^{-1} ~ chi gamma^{-1} I with
// gamma ~ (4 pi a)^{-1} (arXiv:1306.3159 Sec. III.E, eq. Schur_diagonal) is
// kept, and a short-ranged symmetric correction is added:
//   W_ij = D h [ delta_ij 4 pi a0/h + (g(i,j) + g(j,i))/2 ],  |q_j - q_i| < r_c,
// with g a 10 -> 64 -> 64 -> 1 SiLU network of pair features
//   [d/r_c (3), |d|/r_c, frac(q_i/h - 1/2) (3), frac(q_j/h - 1/2) (3)].
// Layers 1 and 2 (and in training the backward products and the weight
// gradients) run on v_mfma_f32_16x16x32_bf16: bfloat16 operands, float32
// accumulation. Layer 3 is a float32 dot product.
//
// MFMA 16x16x32 operand layout (wave64): A is 16 x 32 with lane l holding row
// l & 15, k = 8 (l >> 4) .. + 7; B is 32 x 16 with lane l holding column
// l & 15, k = 8 (l >> 4) .. + 7; the 16 x 16 result gives lane l column l & 15,
// rows 4 (l >> 4) .. + 3.
#include "launch.hpp"

#include <cmath>

namespace brd {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float floatx4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ floatx4 mfma16(const bf16x8& a, const bf16x8& b, const floatx4& c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}

__device__ __forceinline__ float silu_f(float t) { return t / (1.0f + __expf(-t)); }
__device__ __forceinline__ float dsilu_f(float t) {
    const float s = 1.0f / (1.0f + __expf(-t));
    return s * (1.0f + t * (1.0f - s));
}

// Sum over the 16 lanes that share (l >> 4).
__device__ __forceinline__ float sum16(float v) {
    v += __shfl_xor(v, 1, 64);
    v += __shfl_xor(v, 2, 64);
    v += __shfl_xor(v, 4, 64);
    v += __shfl_xor(v, 8, 64);
    return v;
}
// Sum over the 4 lane groups (l >> 4) for a fixed l & 15.
__device__ __forceinline__ float sum_groups(float v) {
    v += __shfl_xor(v, 16, 64);
    v += __shfl_xor(v, 32, 64);
    return v;
}

// ---------------------------------------------------------------------------
// Pair list: blobs binned in a cell grid of edge >= r_c (a single cell when an
// axis has fewer than 3 cells), then each blob scans the neighbouring cells.
__global__ void k_pair_cells(const double* __restrict__ q, int N, PairGeom pg, int* __restrict__ cell_of,
                             int* __restrict__ counts) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= N) return;
    int c[3];
    const int nc[3] = {pg.ncx, pg.ncy, pg.ncz};
    for (int a = 0; a < 3; ++a) {
        const double L = pg.box[a];
        double v = q[3 * i + a];
        v -= L * floor(v / L);
        if (v >= L) v -= L;
        int k = (int)(v / L * nc[a]);
        c[a] = k < 0 ? 0 : (k >= nc[a] ? nc[a] - 1 : k);
    }
    const int id = (c[2] * pg.ncy + c[1]) * pg.ncx + c[0];
    cell_of[i] = id;
    atomicAdd(&counts[id], 1);
}

__device__ __forceinline__ double min_image(double d, double L) { return d - L * rint(d / L); }

template <bool FILL>
__global__ void k_pair_scan(const double* __restrict__ q, int N, PairGeom pg, const int* __restrict__ cell_of,
                            const int* __restrict__ offsets, const int* __restrict__ perm, int* __restrict__ cnt,
                            const int* __restrict__ rowptr, int* __restrict__ col, int* __restrict__ rowidx) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= N) return;
    const int id = cell_of[i];
    const int cx = id % pg.ncx, cy = (id / pg.ncx) % pg.ncy, cz = id / (pg.ncx * pg.ncy);
    const double xi = q[3 * i], yi = q[3 * i + 1], zi = q[3 * i + 2];
    const double rc2 = pg.rc * pg.rc;
    int n = 0;
    const int base = FILL ? rowptr[i] : 0;
    const int dz0 = pg.ncz >= 3 ? -1 : 0, dz1 = pg.ncz >= 3 ? 1 : 0;
    const int dy0 = pg.ncy >= 3 ? -1 : 0, dy1 = pg.ncy >= 3 ? 1 : 0;
    const int dx0 = pg.ncx >= 3 ? -1 : 0, dx1 = pg.ncx >= 3 ? 1 : 0;
    for (int dz = dz0; dz <= dz1; ++dz)
        for (int dy = dy0; dy <= dy1; ++dy)
            for (int dx = dx0; dx <= dx1; ++dx) {
                const int nb = (((cz + dz + pg.ncz) % pg.ncz) * pg.ncy + (cy + dy + pg.ncy) % pg.ncy) * pg.ncx +
                               (cx + dx + pg.ncx) % pg.ncx;
                for (int k = offsets[nb]; k < offsets[nb + 1]; ++k) {
                    const int j = perm[k];
                    const double ddx = min_image(q[3 * j] - xi, pg.box[0]);
                    const double ddy = min_image(q[3 * j + 1] - yi, pg.box[1]);
                    const double ddz = min_image(q[3 * j + 2] - zi, pg.box[2]);
                    if (ddx * ddx + ddy * ddy + ddz * ddz < rc2) {
                        if (FILL) {
                            col[base + n] = j;
                            rowidx[base + n] = i;
                        }
                        ++n;
                    }
                }
            }
    if (!FILL) cnt[i] = n;
}

// Columns of each row in ascending order (fixed order for every later sum).
__global__ void k_row_sort(const int* __restrict__ rowptr, int N, int* __restrict__ col) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= N) return;
    const int lo = rowptr[i], hi = rowptr[i + 1];
    for (int a = lo + 1; a < hi; ++a) {
        const int v = col[a];
        int b = a - 1;
        while (b >= lo && col[b] > v) {
            col[b + 1] = col[b];
            --b;
        }
        col[b + 1] = v;
    }
}

void launch_pair_cells(hipStream_t st, const double* q, int N, PairGeom pg, int* cell_of, int* counts) {
    hipLaunchKernelGGL(k_pair_cells, dim3(nblocks(N)), dim3(kBlock), 0, st, q, N, pg, cell_of, counts);
}
void launch_pair_count(hipStream_t st, const double* q, int N, PairGeom pg, const int* cell_of, const int* offsets,
                       const int* perm, int* cnt) {
    hipLaunchKernelGGL(k_pair_scan<false>, dim3(nblocks(N)), dim3(kBlock), 0, st, q, N, pg, cell_of, offsets, perm,
                       cnt, (const int*)nullptr, (int*)nullptr, (int*)nullptr);
}
void launch_pair_fill(hipStream_t st, const double* q, int N, PairGeom pg, const int* cell_of, const int* offsets,
                      const int* perm, const int* rowptr, int* col, int* rowidx) {
    hipLaunchKernelGGL(k_pair_scan<true>, dim3(nblocks(N)), dim3(kBlock), 0, st, q, N, pg, cell_of, offsets, perm,
                       (int*)nullptr, rowptr, col, rowidx);
    hipLaunchKernelGGL(k_row_sort, dim3(nblocks(N)), dim3(kBlock), 0, st, rowptr, N, col);
}

// rowidx from rowptr after the column sort (entries stay within their row)
__global__ void k_rowidx(const int* __restrict__ rowptr, int N, int* __restrict__ rowidx) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= N) return;
    for (int k = rowptr[i]; k < rowptr[i + 1]; ++k) rowidx[k] = i;
}
void launch_rowidx(hipStream_t st, const int* rowptr, int N, int* rowidx) {
    hipLaunchKernelGGL(k_rowidx, dim3(nblocks(N)), dim3(kBlock), 0, st, rowptr, N, rowidx);
}

// ---------------------------------------------------------------------------
// Pair features of evaluation ev: entry e = ev >> 1, ordering ev & 1.
__device__ __forceinline__ void pair_features(const double* __restrict__ q, PairGeom pg, int a, int b, float* x) {
    double d[3];
    for (int k = 0; k < 3; ++k) {
        double qa = q[3 * a + k], qb = q[3 * b + k];
        const double L = pg.box[k];
        qa -= L * floor(qa / L);
        qb -= L * floor(qb / L);
        d[k] = min_image(qb - qa, L);
        const double sa = qa / pg.h - 0.5, sb = qb / pg.h - 0.5;
        x[4 + k] = (float)(sa - floor(sa));
        x[7 + k] = (float)(sb - floor(sb));
    }
    const double r = sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
    x[0] = (float)(d[0] / pg.rc);
    x[1] = (float)(d[1] / pg.rc);
    x[2] = (float)(d[2] / pg.rc);
    x[3] = (float)(r / pg.rc);
    x[10] = kNuScale * pg.nu[a];
    x[11] = kNuScale * pg.nu[b];
}

// nu_i: the other blobs of row i of the pair list closer than rc / 2 (minimum image, the
// separation formed as in pair_features).
__global__ void k_pair_nu(const double* __restrict__ q, PairGeom pg, const int* __restrict__ rowptr,
                          const int* __restrict__ col, int N, float* __restrict__ nu) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= N) return;
    double qi[3];
    for (int k = 0; k < 3; ++k) {
        const double L = pg.box[k];
        qi[k] = q[3 * i + k] - L * floor(q[3 * i + k] / L);
    }
    int count = 0;
    for (int e = rowptr[i]; e < rowptr[i + 1]; ++e) {
        const int j = col[e];
        if (j == i) continue;
        double r2 = 0.0;
        for (int k = 0; k < 3; ++k) {
            const double L = pg.box[k];
            const double qj = q[3 * j + k] - L * floor(q[3 * j + k] / L);
            const double dk = min_image(qj - qi[k], L);
            r2 += dk * dk;
        }
        if (sqrt(r2) < 0.5 * pg.rc) ++count;
    }
    nu[i] = (float)count;
}

void launch_pair_nu(hipStream_t st, const double* q, PairGeom pg, const int* rowptr, const int* col, int N, float* nu) {
    if (N <= 0) return;
    hipLaunchKernelGGL(k_pair_nu, dim3(nblocks(N)), dim3(kBlock), 0, st, q, pg, rowptr, col, N, nu);
}

// Weight operands in registers (per lane), loaded once per kernel.
struct NetRegs {
    bf16x8 b1[4];       // layer 1 B operand, output tile t
    bf16x8 b2[2][4];    // layer 2 B operand, k step ks, output tile t
    float bias1[4], bias2[4], w3[4];
    float b3;
};

__device__ __forceinline__ void load_net(NetRegs& R, const NetDev& net) {
    const int l = threadIdx.x & 63, c = l & 15, g = l >> 4;
#pragma unroll
    for (int t = 0; t < 4; ++t) {
        bf16x8 v;
#pragma unroll
        for (int j = 0; j < 8; ++j) {
            const int k = 8 * g + j;
            v[j] = k < 16 ? net.W1b[(16 * t + c) * 16 + k] : (__bf16)0.0f;
        }
        R.b1[t] = v;
#pragma unroll
        for (int ks = 0; ks < 2; ++ks) {
            bf16x8 w;
#pragma unroll
            for (int j = 0; j < 8; ++j) w[j] = net.W2b[(16 * t + c) * 64 + 32 * ks + 8 * g + j];
            R.b2[ks][t] = w;
        }
        R.bias1[t] = net.P[kOffB1 + 16 * t + c];
        R.bias2[t] = net.P[kOffB2 + 16 * t + c];
        R.w3[t] = (float)net.w3b[16 * t + c];
    }
    R.b3 = net.P[kOffB3];
}

// Forward of 16 evaluations. feat: this lane's A operand (features of row l&15).
// h1s: wave LDS [16][64] bf16. Outputs (per lane, rows 4g+i): a1, a2, h2 in
// the result layout, g_out (valid on lanes with (l & 15) == 0).
struct Fwd {
    float a1[4][4], a2[4][4], h2[4][4];
    float out[4];
};

__device__ __forceinline__ void net_forward(const NetRegs& R, const bf16x8& feat, __bf16* h1s, Fwd& F) {
    const int l = threadIdx.x & 63, c = l & 15, g = l >> 4;
#pragma unroll
    for (int t = 0; t < 4; ++t) {
        floatx4 acc = {0.f, 0.f, 0.f, 0.f};
        acc = mfma16(feat, R.b1[t], acc);
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const float a = acc[i] + R.bias1[t];
            F.a1[t][i] = a;
            h1s[(4 * g + i) * 64 + 16 * t + c] = (__bf16)silu_f(a);
        }
    }
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    bf16x8 A[2];
#pragma unroll
    for (int ks = 0; ks < 2; ++ks)
#pragma unroll
        for (int j = 0; j < 8; ++j) A[ks][j] = h1s[c * 64 + 32 * ks + 8 * g + j];
    float part[4] = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int t = 0; t < 4; ++t) {
        floatx4 acc = {0.f, 0.f, 0.f, 0.f};
        acc = mfma16(A[0], R.b2[0][t], acc);
        acc = mfma16(A[1], R.b2[1][t], acc);
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const float a = acc[i] + R.bias2[t];
            F.a2[t][i] = a;
            const float hv = silu_f(a);
            F.h2[t][i] = hv;
            part[i] += R.w3[t] * hv;
        }
    }
#pragma unroll
    for (int i = 0; i < 4; ++i) F.out[i] = sum16(part[i]) + R.b3;
}

__device__ __forceinline__ bf16x8 feature_operand(const double* q, PairGeom pg, const int* col, const int* rowidx,
                                                  long long ev, long long nev) {
    const int l = threadIdx.x & 63, g = l >> 4;
    bf16x8 v;
#pragma unroll
    for (int j = 0; j < 8; ++j) v[j] = (__bf16)0.0f;
    if (g < 2) {
        float x[kNetFeat];
        if (ev < nev) {
            const long long e = ev >> 1;
            const int a = rowidx[e], b = col[e];
            if (ev & 1) pair_features(q, pg, b, a, x);
            else pair_features(q, pg, a, b, x);
        } else {
#pragma unroll
            for (int k = 0; k < kNetFeat; ++k) x[k] = 0.f;
        }
#pragma unroll
        for (int j = 0; j < 8; ++j) {
            const int k = 8 * g + j;
            v[j] = (__bf16)(k < kNetFeat ? x[k] : 0.f);
        }
    }
    return v;
}

// W values: one wave per 16 evaluations (8 entries) per pass.
__global__ void __launch_bounds__(kBlock) k_net_assemble(const double* __restrict__ q, PairGeom pg, NetDev net,
                                                         const int* __restrict__ col, const int* __restrict__ rowidx,
                                                         long long nnz, double Dh, double diag,
                                                         double* __restrict__ val) {
    __shared__ __bf16 h1s_all[kBlock / 64][16 * 64];
    const int wv = threadIdx.x >> 6, l = threadIdx.x & 63, c = l & 15, g = l >> 4;
    __bf16* h1s = h1s_all[wv];
    NetRegs R;
    load_net(R, net);
    const long long nev = 2 * nnz;
    const long long ntile = (nev + 15) / 16;
    const long long wglobal = (long long)blockIdx.x * (kBlock / 64) + wv;
    const long long nwaves = (long long)gridDim.x * (kBlock / 64);
    for (long long tile = wglobal; tile < ntile; tile += nwaves) {
        const long long ev0 = tile * 16;
        const bf16x8 feat = feature_operand(q, pg, col, rowidx, ev0 + c, nev);
        Fwd F;
        net_forward(R, feat, h1s, F);
        if (c == 0) {
            // rows 4g .. 4g+3 = evaluations of entries 2g and 2g+1 of this tile
            for (int pr = 0; pr < 2; ++pr) {
                const long long e = (ev0 >> 1) + 2 * g + pr;
                if (e < nnz) {
                    const double gsum = 0.5 * ((double)F.out[2 * pr] + (double)F.out[2 * pr + 1]);
                    val[e] = Dh * (gsum + (rowidx[e] == col[e] ? diag : 0.0));
                }
            }
        }
        __builtin_amdgcn_wave_barrier();
    }
}

void launch_net_assemble(hipStream_t st, const double* q, PairGeom pg, NetDev net, const int* col, const int* rowidx,
                         long long nnz, double Dh, double diag, double* val) {
    const long long tiles = (2 * nnz + 15) / 16;
    long long blocks = (tiles + 3) / 4;
    if (blocks > 2048) blocks = 2048;
    if (blocks < 1) blocks = 1;
    hipLaunchKernelGGL(k_net_assemble, dim3((unsigned)blocks), dim3(kBlock), 0, st, q, pg, net, col, rowidx, nnz, Dh,
                       diag, val);
}

// ---------------------------------------------------------------------------
// CSR SpMV y = W x (FP64), one thread per row, columns ascending.
__global__ void k_spmv(const int* __restrict__ rowptr, const int* __restrict__ col, const double* __restrict__ val,
                       const double* __restrict__ x, double* __restrict__ y, int N) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= N) return;
    double acc = 0.0;
    for (int k = rowptr[i]; k < rowptr[i + 1]; ++k) acc += val[k] * x[col[k]];
    y[i] = acc;
}
void launch_spmv(hipStream_t st, const int* rowptr, const int* col, const double* val, const double* x, double* y,
                 int N) {
    hipLaunchKernelGGL(k_spmv, dim3(nblocks(N)), dim3(kBlock), 0, st, rowptr, col, val, x, y, N);
}

// y = W (x - mean(x)): each block sums x itself (the same order in every block,
// so every block subtracts the same mean), then one thread per row.
__global__ void __launch_bounds__(kBlock) k_spmv_centered(const int* __restrict__ rowptr, const int* __restrict__ col,
                                                          const double* __restrict__ val,
                                                          const double* __restrict__ x, double* __restrict__ y,
                                                          int N) {
    __shared__ double sh[kBlock / 64];
    // the block's copy of mean(x): eight independent partial sums keep eight loads in flight
    double p[8] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    const int bd = (int)blockDim.x;
    int i0 = threadIdx.x;
    for (; i0 + 7 * bd < N; i0 += 8 * bd) {
#pragma unroll
        for (int u = 0; u < 8; ++u) p[u] += x[i0 + u * bd];
    }
    for (; i0 < N; i0 += bd) p[0] += x[i0];
    double s = ((p[0] + p[1]) + (p[2] + p[3])) + ((p[4] + p[5]) + (p[6] + p[7]));
    s = wave_sum(s);
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = s;
    __syncthreads();
    double tot = 0.0;
    for (int w = 0; w < (int)(blockDim.x >> 6); ++w) tot += sh[w];
    const double m = tot / (double)N;
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= N) return;
    double acc = 0.0;
    for (int k = rowptr[i]; k < rowptr[i + 1]; ++k) acc += val[k] * (x[col[k]] - m);
    y[i] = acc;
}

void launch_spmv_centered(hipStream_t st, const int* rowptr, const int* col, const double* val, const double* x,
                          double* y, int N) {
    if (N <= 0) return;
    hipLaunchKernelGGL(k_spmv_centered, dim3(nblocks(N)), dim3(kBlock), 0, st, rowptr, col, val, x, y, N);
}

// Non-finite entries of W (watchdog)
__global__ void __launch_bounds__(kFinBlock) k_count_bad(const double* v, long long n, int* out) {
    int bad = 0;
    for (long long i = threadIdx.x; i < n; i += blockDim.x) bad += !(v[i] == v[i] && v[i] - v[i] == 0.0);
    __shared__ int sh[kFinBlock];
    sh[threadIdx.x] = bad;
    __syncthreads();
    if (threadIdx.x == 0) {
        int s = 0;
        for (int t = 0; t < (int)blockDim.x; ++t) s += sh[t];
        out[0] = s;
    }
}
void launch_count_bad(hipStream_t st, const double* v, long long n, int* out) {
    hipLaunchKernelGGL(k_count_bad, dim3(1), dim3(kFinBlock), 0, st, v, n, out);
}

// ---------------------------------------------------------------------------
// Training.
//
// GW_e = sum_s c_s rp_s[row e] yp_s[col e] with c_s = 2 / (S |x_s|^2); the
// network output gradient of both evaluations of entry e is D h GW_e / 2.
__global__ void k_entry_grad(const int* __restrict__ rowidx, const int* __restrict__ col, long long nnz,
                             const double* __restrict__ RP, const double* __restrict__ YP,
                             const double* __restrict__ coef, int S, int N, double half_Dh, float* __restrict__ dg) {
    const long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= nnz) return;
    const int i = rowidx[e], j = col[e];
    double acc = 0.0;
    for (int s = 0; s < S; ++s) acc += coef[s] * RP[(size_t)s * N + i] * YP[(size_t)s * N + j];
    dg[e] = (float)(half_Dh * acc);
}
void launch_entry_grad(hipStream_t st, const int* rowidx, const int* col, long long nnz, const double* RP,
                       const double* YP, const double* coef, int S, int N, double half_Dh, float* dg) {
    hipLaunchKernelGGL(k_entry_grad, dim3((unsigned)((nnz + kBlock - 1) / kBlock)), dim3(kBlock), 0, st, rowidx, col,
                       nnz, RP, YP, coef, S, N, half_Dh, dg);
}

// Per-wave gradient partials: one slot of kNetParams floats per wave.
// Each wave walks tiles of 32 evaluations (two 16-row halves): forward,
// backward to the pre-activations, then weight gradients as MFMA products
// with the 32 evaluations as the contraction dimension.
__global__ void __launch_bounds__(kBlock) k_net_backward(const double* __restrict__ q, PairGeom pg, NetDev net,
                                                         const int* __restrict__ col, const int* __restrict__ rowidx,
                                                         long long nnz, const float* __restrict__ dg,
                                                         float* __restrict__ wpart) {
    struct WaveLds {
        __bf16 h1[32 * 64];
        __bf16 da2[32 * 64];
        __bf16 da1[32 * 64];
        __bf16 x[32 * 16];
    };
    __shared__ WaveLds lds_all[kBlock / 64];
    const int wv = threadIdx.x >> 6, l = threadIdx.x & 63, c = l & 15, g = l >> 4;
    WaveLds& S = lds_all[wv];
    NetRegs R;
    load_net(R, net);
    // W2 as a B operand of d_h1 = d_a2 . W2: B[k = o2][col = k1] = W2[o2][k1]
    bf16x8 w2t[2][4];
#pragma unroll
    for (int ks = 0; ks < 2; ++ks)
#pragma unroll
        for (int t = 0; t < 4; ++t)
#pragma unroll
            for (int j = 0; j < 8; ++j) w2t[ks][t][j] = net.W2b[(32 * ks + 8 * g + j) * 64 + 16 * t + c];
    floatx4 gW2[4][4];
    floatx4 gW1[4];
#pragma unroll
    for (int a = 0; a < 4; ++a) {
        gW1[a] = floatx4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int b = 0; b < 4; ++b) gW2[a][b] = floatx4{0.f, 0.f, 0.f, 0.f};
    }
    float gb1[4] = {0, 0, 0, 0}, gb2[4] = {0, 0, 0, 0}, gw3[4] = {0, 0, 0, 0}, gb3 = 0.f;
    const long long nev = 2 * nnz;
    const long long ntile = (nev + 31) / 32;
    const long long wglobal = (long long)blockIdx.x * (kBlock / 64) + wv;
    const long long nwaves = (long long)gridDim.x * (kBlock / 64);
    for (long long tile = wglobal; tile < ntile; tile += nwaves) {
#pragma unroll
        for (int half = 0; half < 2; ++half) {
            const long long ev0 = tile * 32 + 16 * half;
            const bf16x8 feat = feature_operand(q, pg, col, rowidx, ev0 + c, nev);
            // keep the features (rows = evaluations) for the W1 gradient
            if (g < 2)
#pragma unroll
                for (int j = 0; j < 8; ++j) S.x[(16 * half + c) * 16 + 8 * g + j] = feat[j];
            Fwd F;
            net_forward(R, feat, S.h1 + 16 * half * 64, F);
            // output gradient of rows 4g+i (evaluation ev0 + 4g + i)
            float dout[4];
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const long long ev = ev0 + 4 * g + i;
                dout[i] = ev < nev ? dg[ev >> 1] : 0.f;
            }
            float da2[4][4];
#pragma unroll
            for (int t = 0; t < 4; ++t)
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    gw3[t] += dout[i] * F.h2[t][i];
                    da2[t][i] = dout[i] * R.w3[t] * dsilu_f(F.a2[t][i]);
                    gb2[t] += da2[t][i];
                    S.da2[(16 * half + 4 * g + i) * 64 + 16 * t + c] = (__bf16)da2[t][i];
                }
            if (c == 0)
#pragma unroll
                for (int i = 0; i < 4; ++i) gb3 += dout[i];
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            // d_h1 = d_a2 . W2 (A = d_a2 rows of this half)
            bf16x8 A[2];
#pragma unroll
            for (int ks = 0; ks < 2; ++ks)
#pragma unroll
                for (int j = 0; j < 8; ++j) A[ks][j] = S.da2[(16 * half + c) * 64 + 32 * ks + 8 * g + j];
#pragma unroll
            for (int t = 0; t < 4; ++t) {
                floatx4 acc = {0.f, 0.f, 0.f, 0.f};
                acc = mfma16(A[0], w2t[0][t], acc);
                acc = mfma16(A[1], w2t[1][t], acc);
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    const float d1 = acc[i] * dsilu_f(F.a1[t][i]);
                    gb1[t] += d1;
                    S.da1[(16 * half + 4 * g + i) * 64 + 16 * t + c] = (__bf16)d1;
                }
            }
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        }
        // weight gradients, contraction over the 32 evaluations of the tile:
        // gW2[o][k] += sum_ev da2[ev][o] h1[ev][k], gW1[o][k] += sum_ev da1[ev][o] x[ev][k]
#pragma unroll
        for (int to = 0; to < 4; ++to) {
            bf16x8 A2, A1;
#pragma unroll
            for (int j = 0; j < 8; ++j) {
                A2[j] = S.da2[(8 * g + j) * 64 + 16 * to + c];
                A1[j] = S.da1[(8 * g + j) * 64 + 16 * to + c];
            }
#pragma unroll
            for (int tk = 0; tk < 4; ++tk) {
                bf16x8 B;
#pragma unroll
                for (int j = 0; j < 8; ++j) B[j] = S.h1[(8 * g + j) * 64 + 16 * tk + c];
                gW2[to][tk] = mfma16(A2, B, gW2[to][tk]);
            }
            bf16x8 Bx;
#pragma unroll
            for (int j = 0; j < 8; ++j) Bx[j] = S.x[(8 * g + j) * 16 + c];
            gW1[to] = mfma16(A1, Bx, gW1[to]);
        }
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    }
    // write this wave's partial gradient (W1 cols < 10 only)
    float* out = wpart + (size_t)wglobal * kNetParams;
#pragma unroll
    for (int to = 0; to < 4; ++to)
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int o = 16 * to + 4 * g + i;
            if (c < kNetFeat) out[kOffW1 + o * kNetFeat + c] = gW1[to][i];
#pragma unroll
            for (int tk = 0; tk < 4; ++tk) out[kOffW2 + o * 64 + 16 * tk + c] = gW2[to][tk][i];
        }
#pragma unroll
    for (int t = 0; t < 4; ++t) {
        const float b1 = sum_groups(gb1[t]), b2 = sum_groups(gb2[t]), w3 = sum_groups(gw3[t]);
        if (g == 0) {
            out[kOffB1 + 16 * t + c] = b1;
            out[kOffB2 + 16 * t + c] = b2;
            out[kOffW3 + 16 * t + c] = w3;
        }
    }
    float b3 = gb3;
    b3 += __shfl_xor(b3, 16, 64);
    b3 += __shfl_xor(b3, 32, 64);
    if (l == 0) out[kOffB3] = b3;
}

int launch_net_backward(hipStream_t st, const double* q, PairGeom pg, NetDev net, const int* col, const int* rowidx,
                        long long nnz, const float* dg, float* wpart, int max_waves) {
    const long long tiles = (2 * nnz + 31) / 32;
    long long waves = tiles < max_waves ? tiles : max_waves;
    if (waves < 4) waves = 4;
    const long long blocks = (waves + 3) / 4;
    hipLaunchKernelGGL(k_net_backward, dim3((unsigned)blocks), dim3(kBlock), 0, st, q, pg, net, col, rowidx, nnz, dg,
                       wpart);
    return (int)(blocks * 4);
}

// grad += sum over waves (fixed order), one thread per parameter
__global__ void k_grad_reduce(const float* __restrict__ wpart, int nwaves, float* __restrict__ grad) {
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= kNetParams) return;
    float s = 0.f;
    for (int w = 0; w < nwaves; ++w) s += wpart[(size_t)w * kNetParams + p];
    grad[p] += s;
}
void launch_grad_reduce(hipStream_t st, const float* wpart, int nwaves, float* grad) {
    hipLaunchKernelGGL(k_grad_reduce, dim3(nblocks(kNetParams)), dim3(kBlock), 0, st, wpart, nwaves, grad);
}

// Adam (Kingma and Ba, 2015) on float32 masters, then refresh the bf16 copies.
__global__ void k_adam(float* __restrict__ P, float* __restrict__ m, float* __restrict__ v,
                       const float* __restrict__ grad, float lr, float b1, float b2, float eps, float c1, float c2) {
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= kNetParams) return;
    const float g = grad[p];
    const float mm = b1 * m[p] + (1.f - b1) * g;
    const float vv = b2 * v[p] + (1.f - b2) * g * g;
    m[p] = mm;
    v[p] = vv;
    P[p] -= lr * (mm / c1) / (sqrtf(vv / c2) + eps);
}
void launch_adam(hipStream_t st, float* P, float* m, float* v, const float* grad, float lr, float b1, float b2,
                 float eps, int t) {
    const float c1 = 1.f - powf(b1, (float)t), c2 = 1.f - powf(b2, (float)t);
    hipLaunchKernelGGL(k_adam, dim3(nblocks(kNetParams)), dim3(kBlock), 0, st, P, m, v, grad, lr, b1, b2, eps, c1,
                       c2);
}

__global__ void k_net_pack(const float* __restrict__ P, __bf16* __restrict__ W1b, __bf16* __restrict__ W2b,
                           __bf16* __restrict__ w3b) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t < 64 * 16) {
        const int o = t / 16, k = t % 16;
        W1b[t] = (__bf16)(k < kNetFeat ? P[kOffW1 + o * kNetFeat + k] : 0.f);
    }
    if (t < 64 * 64) W2b[t] = (__bf16)P[kOffW2 + t];
    if (t < 64) w3b[t] = (__bf16)P[kOffW3 + t];
}
void launch_net_pack(hipStream_t st, const float* P, __bf16* W1b, __bf16* W2b, __bf16* w3b) {
    hipLaunchKernelGGL(k_net_pack, dim3(16), dim3(kBlock), 0, st, P, W1b, W2b, w3b);
}

}  // namespace brd
