// Blob kernels: placement and binning, local averaging J, spreading S, and
// the N-vector kernels of the Schur-complement GMRES.
//
// arXiv:1306.3159 Sec. III.A: (J c)_i = sum_k phi_w(q_i - r_k) c_k with the
// tensor-product kernel of eq. tensor_product, and S = h^-3 J^T. The kernels
// are Peskin's four-point function and the three-point function of Roma,
// Peskin and Berger (the paper states their moment conditions, eq.
// JS_invariance, and cites these forms).
//
// Spreading is a gather: one work-group per grid tile collects the blobs
// binned in its own and neighbouring tiles, stages their weights in LDS and
// lets each thread sum the contributions to the cells it owns, in a fixed
// order. No atomics touch floating-point data, so results are bitwise
// reproducible.
#include "launch.hpp"

#include <cmath>

namespace brd {

__device__ __forceinline__ double kern4(double r) {
    const double a = fabs(r);
    if (a <= 1.0) return (3.0 - 2.0 * a + sqrt(fmax(1.0 + 4.0 * a * (1.0 - a), 0.0))) * 0.125;
    if (a < 2.0) return (5.0 - 2.0 * a - sqrt(fmax(-7.0 + a * (12.0 - 4.0 * a), 0.0))) * 0.125;
    return 0.0;
}

__device__ __forceinline__ double kern3(double r) {
    const double a = fabs(r);
    if (a <= 0.5) return (1.0 + sqrt(fmax(1.0 - 3.0 * a * a, 0.0))) * (1.0 / 3.0);
    if (a < 1.5) {
        const double b = 1.0 - a;
        return (5.0 - 3.0 * a - sqrt(fmax(1.0 - 3.0 * b * b, 0.0))) * (1.0 / 6.0);
    }
    return 0.0;
}

// ---------------------------------------------------------------------------
// Placement: wrap q into the box, first support cell k0 (w = 4: floor(s) - 1,
// w = 3: nearest cell - 1, with s = q/h - 1/2), the w weights per axis
// (zero-padded to 4) and the tile of the bin cell k0 + 1.
__global__ void k_blob_setup(const double* __restrict__ q, int N, BlobGeom g, int* __restrict__ base,
                             double* __restrict__ wts, int* __restrict__ tile_of, int* __restrict__ counts) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= N) return;
    const int n[3] = {g.nx, g.ny, g.nz};
    const int te[3] = {g.tx, g.ty, g.tz};
    int tc[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const double Lb = n[a] * g.h;
        double qa = q[3 * i + a];
        qa -= Lb * floor(qa / Lb);
        if (qa >= Lb) qa -= Lb;
        const double s = qa / g.h - 0.5;
        const int k0 = (g.w == 4) ? (int)floor(s) - 1 : (int)floor(s + 0.5) - 1;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const double d = s - (double)(k0 + j);
            wts[(3 * i + a) * 4 + j] = (j < g.w) ? (g.w == 4 ? kern4(d) : kern3(d)) : 0.0;
        }
        const int kb = ((k0 % n[a]) + n[a]) % n[a];
        base[3 * i + a] = kb;
        const int bin = kb + 1 == n[a] ? 0 : kb + 1;
        tc[a] = bin / te[a];
    }
    const int t = (tc[2] * g.nty + tc[1]) * g.ntx + tc[0];
    tile_of[i] = t;
    atomicAdd(&counts[t], 1);
}

void launch_blob_setup(hipStream_t st, const double* q, int N, BlobGeom g, int* base, double* wts, int* tile_of,
                       int* counts) {
    if (N <= 0) return;
    hipLaunchKernelGGL(k_blob_setup, dim3(nblocks(N)), dim3(kBlock), 0, st, q, N, g, base, wts, tile_of, counts);
}

// Exclusive scan of bin counts, one work-group, contiguous chunk per thread.
__global__ void __launch_bounds__(kFinBlock) k_bin_scan(const int* __restrict__ counts, int nt, int* offsets) {
    __shared__ int sh[kFinBlock];
    const int per = (nt + blockDim.x - 1) / blockDim.x;
    const int lo = threadIdx.x * per, hi = min(lo + per, nt);
    int s = 0;
    for (int i = lo; i < hi; ++i) s += counts[i];
    sh[threadIdx.x] = s;
    __syncthreads();
    if (threadIdx.x == 0) {
        int run = 0;
        for (int t = 0; t < (int)blockDim.x; ++t) {
            const int v = sh[t];
            sh[t] = run;
            run += v;
        }
        offsets[nt] = run;
    }
    __syncthreads();
    int run = sh[threadIdx.x];
    for (int i = lo; i < hi; ++i) {
        offsets[i] = run;
        run += counts[i];
    }
}

void launch_bin_scan(hipStream_t st, const int* counts, int ntiles, int* offsets) {
    hipLaunchKernelGGL(k_bin_scan, dim3(1), dim3(kFinBlock), 0, st, counts, ntiles, offsets);
}

__global__ void k_bin_scatter(const int* __restrict__ tile_of, int N, const int* __restrict__ offsets, int* cursor,
                              int* perm) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= N) return;
    const int t = tile_of[i];
    perm[offsets[t] + atomicAdd(&cursor[t], 1)] = i;
}

void launch_bin_scatter(hipStream_t st, const int* tile_of, int N, const int* offsets, int* cursor, int* perm) {
    if (N <= 0) return;
    hipLaunchKernelGGL(k_bin_scatter, dim3(nblocks(N)), dim3(kBlock), 0, st, tile_of, N, offsets, cursor, perm);
}

// Within each bin, order blobs by index so that every later sum is in a fixed order.
__global__ void k_bin_sort(const int* __restrict__ offsets, int nt, int* perm) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= nt) return;
    const int lo = offsets[t], hi = offsets[t + 1];
    for (int a = lo + 1; a < hi; ++a) {
        const int v = perm[a];
        int b = a - 1;
        while (b >= lo && perm[b] > v) {
            perm[b + 1] = perm[b];
            --b;
        }
        perm[b + 1] = v;
    }
}

void launch_bin_sort(hipStream_t st, const int* offsets, int ntiles, int* perm) {
    hipLaunchKernelGGL(k_bin_sort, dim3(nblocks(ntiles)), dim3(kBlock), 0, st, offsets, ntiles, perm);
}

// ---------------------------------------------------------------------------
// Local averaging: one wave64 per blob, lane l <-> support cell
// (l & 3, (l >> 2) & 3, l >> 4); a wave reduction sums the 64 products.
// Blobs are visited in tile order so neighbouring waves share cache lines.
__device__ __forceinline__ void interp_body(const double* __restrict__ x, int N, const BlobGeom& g,
                                            const int* __restrict__ base, const double* __restrict__ wts,
                                            const int* __restrict__ perm, double* __restrict__ jx,
                                            const double* __restrict__ kappa, double* __restrict__ out, Blk blk) {
    const int wv = blk.b * (blockDim.x >> 6) + (threadIdx.x >> 6);
    if (wv >= N) return;
    const int i = perm[wv];
    const int l = threadIdx.x & 63;
    const int a = l & 3, b = (l >> 2) & 3, c = l >> 4;
    int cx = base[3 * i] + a, cy = base[3 * i + 1] + b, cz = base[3 * i + 2] + c;
    cx = cx >= g.nx ? cx - g.nx : cx;
    cy = cy >= g.ny ? cy - g.ny : cy;
    cz = cz >= g.nz ? cz - g.nz : cz;
    const double* w = wts + (size_t)i * 12;
    const double wgt = w[a] * w[4 + b] * w[8 + c];
    double v = wgt * x[((size_t)cz * g.ny + cy) * g.nx + cx];
    v = wave_sum(v);
    if (l == 0) {
        if (jx) jx[i] = v;
        if (out) out[i] = kappa ? kappa[i] * v : v;
    }
}

__global__ void __launch_bounds__(kBlock) k_interp(const double* __restrict__ x, int N, BlobGeom g,
                                                   const int* __restrict__ base, const double* __restrict__ wts,
                                                   const int* __restrict__ perm, double* __restrict__ jx,
                                                   const double* __restrict__ kappa, double* __restrict__ out,
                                                   const Scalars* sc) {
    if (sc && sc->done) return;
    interp_body(x, N, g, base, wts, perm, jx, kappa, out, Blk{blockIdx.x, gridDim.x});
}

void launch_interp(hipStream_t st, const double* x, int N, BlobGeom g, const int* base, const double* wts,
                   const int* perm, double* jx, const double* kappa, double* out, const Scalars* sc) {
    if (N <= 0) return;
    const int per = kBlock / 64;
    hipLaunchKernelGGL(k_interp, dim3((N + per - 1) / per), dim3(kBlock), 0, st, x, N, g, base, wts, perm, jx, kappa,
                       out, sc);
}

// out_i = (J z)_i for z in a red/black split level-0 layout (u0, u1 of type T):
// the same weights and summation order as interp_body on the natural copy of z.
template <typename T>
__global__ void __launch_bounds__(kBlock) k_interp_split(const T* __restrict__ z0, const T* __restrict__ z1, int N,
                                                         BlobGeom g, const int* __restrict__ base,
                                                         const double* __restrict__ wts, const int* __restrict__ perm,
                                                         double* __restrict__ out) {
    const int wv = blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
    if (wv >= N) return;
    const int i = perm[wv];
    const int l = threadIdx.x & 63;
    const int a = l & 3, b = (l >> 2) & 3, c = l >> 4;
    int cx = base[3 * i] + a, cy = base[3 * i + 1] + b, cz = base[3 * i + 2] + c;
    cx = cx >= g.nx ? cx - g.nx : cx;
    cy = cy >= g.ny ? cy - g.ny : cy;
    cz = cz >= g.nz ? cz - g.nz : cz;
    const double* w = wts + (size_t)i * 12;
    const double wgt = w[a] * w[4 + b] * w[8 + c];
    double v = wgt * split_at(z0, z1, cx, cy, cz, g.nx >> 1, g.ny);
    v = wave_sum(v);
    if (l == 0) out[i] = v;
}

template <typename T>
void launch_interp_split(hipStream_t st, const T* z0, const T* z1, int N, BlobGeom g, const int* base,
                         const double* wts, const int* perm, double* out) {
    if (N <= 0) return;
    const int per = kBlock / 64;
    hipLaunchKernelGGL(k_interp_split<T>, dim3((N + per - 1) / per), dim3(kBlock), 0, st, z0, z1, N, g, base, wts,
                       perm, out);
}
template void launch_interp_split<float>(hipStream_t, const float*, const float*, int, BlobGeom, const int*,
                                         const double*, const int*, double*);
template void launch_interp_split<double>(hipStream_t, const double*, const double*, int, BlobGeom, const int*,
                                          const double*, const int*, double*);

// Batched blob term of B = alpha I - D L + S kappa J inside a CG iteration:
// jx = J p, mu = kappa jx (interp), then q += h^-3 S mu (spread, touched cells only).
__global__ void __launch_bounds__(kBlock) kb_interp(const InstDev* inst, const int* gate, const BatchTab* tab) {
    const BatchEntry* ent = tab_entries(tab);
    for (unsigned g = blockIdx.x; g < tab->total; g += gridDim.x) {
        Blk blk;
        const InstDev* I = batch_slot(inst, gate, ent, tab->n, g, blk);
        if (!I || !I->blobs) continue;
        interp_body(I->p, I->N, I->geom, I->base, I->wts, I->perm, I->jx, I->kappa, I->mu, blk);
    }
}

// sum_e w[e] m(blob[e]) over the entries of touched cell k
__device__ __forceinline__ double spread_acc(int k, const SpreadLists& L, const SpreadMult& M) {
    double acc = 0.0;
    for (int e = L.ptr[k]; e < L.ptr[k + 1]; ++e) {
        const int b = L.blob[e];
        double v = M.lam ? M.lam[b] : 0.0;
        if (M.lam2) v += M.c2 * M.lam2[b];
        acc += L.w[e] * (v + M.shift);
    }
    return acc;
}

// out[c] = base(c) + scale * sum_e w[e] m(blob[e]) for touched cell k
__device__ __forceinline__ void spread_sparse_cell(int k, const SpreadLists& L, const SpreadMult& M,
                                                   const double* base_in, double* out, double scale) {
    const double acc = spread_acc(k, L, M);
    const int c = L.cell[k];
    const double b = base_in ? base_in[c] : 0.0;
    out[c] = b + scale * acc;
}

// q += S mu on the touched cells of every gated instance
__global__ void __launch_bounds__(kBlock) kb_spread(const InstDev* inst, const int* gate, const BatchTab* tab) {
    const BatchEntry* ent = tab_entries(tab);
    for (unsigned g = blockIdx.x; g < tab->total; g += gridDim.x) {
        Blk blk;
        const InstDev* I = batch_slot(inst, gate, ent, tab->n, g, blk);
        if (!I || !I->blobs) continue;
        const int k = (int)(blk.b * blockDim.x + threadIdx.x);
        if (k < I->ntouched)
            spread_sparse_cell(k, SpreadLists{I->ntouched, I->tcell, I->tptr, I->tblob, I->tw},
                               SpreadMult{I->mu, nullptr, 0.0, 0.0}, I->q, I->q, I->inv_h3);
    }
}

void launchb_blob(hipStream_t st, int spread, const InstDev* inst, const int* gate, const BatchTab* tab,
                  unsigned grid) {
    if (spread) hipLaunchKernelGGL(kb_spread, dim3(grid), dim3(kBlock), 0, st, inst, gate, tab);
    else hipLaunchKernelGGL(kb_interp, dim3(grid), dim3(kBlock), 0, st, inst, gate, tab);
}


// ---------------------------------------------------------------------------
// Spreading from contribution lists. The blob placement is fixed for a handle,
// so the weights one tile gather would find for each cell can be listed once:
// per touched cell, the (blob, weight) pairs with a nonzero weight, in the
// gather's candidate order (neighbour tiles z-major, each tile's blobs in bin
// order) and with the gather's product order ((wx wy) wz) lam. A spread is
// then a dense pass (zero or copy of the base) plus one thread per touched
// cell, and the sums are bitwise those of the gather.
//
// k_spread_plan, one work-group per tile: mode 0 counts the tile's entries and
// touched cells into cnt[t] and cnt[ntiles + t]; mode 1 writes them at the
// scanned offsets offE[t], offC[t] (tcell: cell index, tptr: first entry).
__global__ void __launch_bounds__(kBlock) k_spread_plan(int mode, BlobGeom g, const int* __restrict__ base,
                                                        const double* __restrict__ wts,
                                                        const int* __restrict__ offsets, const int* __restrict__ perm,
                                                        int* __restrict__ cnt, const int* __restrict__ offE,
                                                        const int* __restrict__ offC, int* __restrict__ tcell,
                                                        int* __restrict__ tptr, int* __restrict__ tblob,
                                                        double* __restrict__ tw) {
    struct Cand {
        int bx, by, bz, i;
        double w[12];
    };
    __shared__ Cand stg[kStageBlobs];
    __shared__ int rng_lo[27], rng_pre[28], nb_lo[27], nb_len[27];
    __shared__ int nrng;
    __shared__ int ncount[2 * kBlock], nstart[2 * kBlock + 1], crank[2 * kBlock + 1];
    const int ntiles = g.ntx * g.nty * g.ntz;
    const int t = blockIdx.x;
    const int tix = t % g.ntx, tiy = (t / g.ntx) % g.nty, tiz = t / (g.ntx * g.nty);
    if (threadIdx.x < 27) {
        const int d = threadIdx.x;
        const int dx = d % 3 - 1, dy = (d / 3) % 3 - 1, dz = d / 9 - 1;
        const int vx = (tix + dx + g.ntx) % g.ntx, vy = (tiy + dy + g.nty) % g.nty, vz = (tiz + dz + g.ntz) % g.ntz;
        bool first = true;
        for (int e = -1; e < dx; ++e) first &= (tix + e + g.ntx) % g.ntx != vx;
        for (int e = -1; e < dy; ++e) first &= (tiy + e + g.nty) % g.nty != vy;
        for (int e = -1; e < dz; ++e) first &= (tiz + e + g.ntz) % g.ntz != vz;
        int lo = 0, len = 0;
        if (first) {
            const int nt = (vz * g.nty + vy) * g.ntx + vx;
            lo = offsets[nt];
            len = offsets[nt + 1] - lo;
        }
        nb_lo[d] = lo;
        nb_len[d] = len;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        int nr = 0, pre = 0;
        for (int d = 0; d < 27; ++d)
            if (nb_len[d] > 0) {
                rng_lo[nr] = nb_lo[d];
                rng_pre[nr] = pre;
                pre += nb_len[d];
                ++nr;
            }
        rng_pre[nr] = pre;
        nrng = nr;
    }
    __syncthreads();
    const int K = rng_pre[nrng];
    const int tcells = g.tx * g.ty * g.tz;
    int cell[2][3];
    int n[2] = {0, 0};
#pragma unroll
    for (int e = 0; e < 2; ++e) {
        const int lc = threadIdx.x + e * blockDim.x;
        const int lx = lc % g.tx, ly = (lc / g.tx) % g.ty, lz = lc / (g.tx * g.ty);
        cell[e][0] = tix * g.tx + lx;
        cell[e][1] = tiy * g.ty + ly;
        cell[e][2] = tiz * g.tz + lz;
    }
    // pass 0 counts per cell; pass 1 (mode 1) writes at the per-cell starts
    for (int pass = 0; pass <= mode; ++pass) {
        int cur[2] = {0, 0};
        if (pass == 1) {
#pragma unroll
            for (int e = 0; e < 2; ++e) cur[e] = offE[t] + nstart[threadIdx.x + e * blockDim.x];
        }
        for (int c0 = 0; c0 < K; c0 += kStageBlobs) {
            const int cn = min(kStageBlobs, K - c0);
            __syncthreads();
            if ((int)threadIdx.x < cn) {
                const int k = c0 + threadIdx.x;
                int r = 0;
                while (rng_pre[r + 1] <= k) ++r;
                const int i = perm[rng_lo[r] + (k - rng_pre[r])];
                Cand c;
                c.bx = base[3 * i];
                c.by = base[3 * i + 1];
                c.bz = base[3 * i + 2];
                c.i = i;
#pragma unroll
                for (int j = 0; j < 12; ++j) c.w[j] = wts[(size_t)i * 12 + j];
                stg[threadIdx.x] = c;
            }
            __syncthreads();
#pragma unroll
            for (int e = 0; e < 2; ++e) {
                const int lc = threadIdx.x + e * blockDim.x;
                if (lc >= tcells) continue;
                for (int j = 0; j < cn; ++j) {
                    int a = cell[e][0] - stg[j].bx;
                    int b = cell[e][1] - stg[j].by;
                    int c = cell[e][2] - stg[j].bz;
                    a += a < 0 ? g.nx : 0;
                    b += b < 0 ? g.ny : 0;
                    c += c < 0 ? g.nz : 0;
                    if (a < 4 && b < 4 && c < 4) {
                        const double wv = stg[j].w[a] * stg[j].w[4 + b] * stg[j].w[8 + c];
                        if (wv != 0.0) {
                            if (pass == 1) {
                                tblob[cur[e]] = stg[j].i;
                                tw[cur[e]] = wv;
                                ++cur[e];
                            } else {
                                ++n[e];
                            }
                        }
                    }
                }
            }
        }
        if (pass == 0) {
#pragma unroll
            for (int e = 0; e < 2; ++e) ncount[threadIdx.x + e * blockDim.x] = n[e];
            __syncthreads();
            if (threadIdx.x == 0) {
                int se = 0, sc = 0;
                for (int lc = 0; lc < tcells; ++lc) {
                    nstart[lc] = se;
                    crank[lc] = sc;
                    se += ncount[lc];
                    sc += ncount[lc] > 0 ? 1 : 0;
                }
                nstart[tcells] = se;
                crank[tcells] = sc;
                if (mode == 0) {
                    cnt[t] = se;
                    cnt[ntiles + t] = sc;
                }
            }
            __syncthreads();
            if (mode == 1) {
#pragma unroll
                for (int e = 0; e < 2; ++e) {
                    const int lc = threadIdx.x + e * blockDim.x;
                    if (lc < tcells && ncount[lc] > 0) {
                        const int slot = offC[t] + crank[lc];
                        tcell[slot] = (cell[e][2] * g.ny + cell[e][1]) * g.nx + cell[e][0];
                        tptr[slot] = offE[t] + nstart[lc];
                    }
                }
                if (t == ntiles - 1 && threadIdx.x == 0) tptr[offC[ntiles]] = offE[ntiles];
            }
        }
    }
}

void launch_spread_plan(hipStream_t st, int mode, BlobGeom g, const int* base, const double* wts, const int* offsets,
                        const int* perm, int* cnt, const int* offE, const int* offC, int* tcell, int* tptr,
                        int* tblob, double* tw) {
    const unsigned nt = (unsigned)g.ntx * g.nty * g.ntz;
    hipLaunchKernelGGL(k_spread_plan, dim3(nt), dim3(kBlock), 0, st, mode, g, base, wts, offsets, perm, cnt, offE, offC,
                       tcell, tptr, tblob, tw);
}

// out[c] = base(c) + scale * sum_e w[e] m(blob[e]) over the touched cells c
// (base(c) = base_in[c], 0 without base_in); other cells are not touched (the
// caller's dense pass set them, or base_in aliases out).
__global__ void __launch_bounds__(kBlock) k_spread_sparse(SpreadLists L, SpreadMult M, const double* base_in,
                                                          double* out, double scale, const Scalars* sc) {
    if (sc && sc->done) return;
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= L.n) return;
    spread_sparse_cell(k, L, M, base_in, out, scale);
}

void launch_spread_sparse(hipStream_t st, const SpreadLists& L, const SpreadMult& M, const double* base_in,
                          double* out, double scale, const Scalars* sc) {
    if (L.n <= 0) return;
    hipLaunchKernelGGL(k_spread_sparse, dim3(nblocks(L.n)), dim3(kBlock), 0, st, L, M, base_in, out, scale, sc);
}

// V-cycle entry at the touched cells: r = base(c) + scale S m, the split
// level-0 copy f and the first red half-sweep from zero (u_red = f_red / diag)
// are written there only. Without base_in the caller has zeroed u0 (and f0, f1
// unless they hold zeros outside the touched cells from a previous entry of the
// same lists); with base_in, k_enter of base_in has set every other cell.
// Bitwise the spread into a grid followed by k_enter.
template <typename T>
__global__ void __launch_bounds__(kBlock) k_spread_enter(SpreadLists L, SpreadMult M, const double* __restrict__ base_in,
                                                         double scale, T* __restrict__ f0, T* __restrict__ f1,
                                                         T* __restrict__ u0, int nx, int ny, double inv_diag) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= L.n) return;
    const double acc = spread_acc(k, L, M);
    const int c = L.cell[k];
    const double r = (base_in ? base_in[c] : 0.0) + scale * acc;
    const int X = c % nx;
    const int t = c / nx;
    const int Y = t % ny, Z = t / ny;
    const size_t j = ((size_t)Z * ny + Y) * (nx >> 1) + (X >> 1);
    if ((X + Y + Z) & 1) {
        f1[j] = (T)r;
    } else {
        f0[j] = (T)r;
        if (u0) u0[j] = (T)((T)r * (T)inv_diag);  // null: the cycle opens from f
    }
}

template <typename T>
void launch_spread_enter(hipStream_t st, const SpreadLists& L, const SpreadMult& M, const double* base_in,
                         double scale, T* f0, T* f1, T* u0, int nx, int ny, double inv_diag) {
    if (L.n <= 0) return;
    hipLaunchKernelGGL(k_spread_enter<T>, dim3(nblocks(L.n)), dim3(kBlock), 0, st, L, M, base_in, scale, f0, f1, u0,
                       nx, ny, inv_diag);
}
template void launch_spread_enter<float>(hipStream_t, const SpreadLists&, const SpreadMult&, const double*, double,
                                         float*, float*, float*, int, int, double);
template void launch_spread_enter<double>(hipStream_t, const SpreadLists&, const SpreadMult&, const double*, double,
                                          double*, double*, double*, int, int, double);

// The entry from the residual of a split-layout guess c at the touched cells of a spread term:
// r = (g - (alpha c - D L c)) + scale S m, f and (u0 set) the red zero-guess sweep written
// there only, after k_resid_enter has written every cell.
template <typename T>
__global__ void __launch_bounds__(kBlock) k_resid_spread_enter(SpreadLists L, SpreadMult M,
                                                               const double* __restrict__ g, const T* __restrict__ c0,
                                                               const T* __restrict__ c1, double scale,
                                                               T* __restrict__ f0, T* __restrict__ f1,
                                                               T* __restrict__ u0, int nx, int ny, int nz, double alpha,
                                                               double s, double inv_diag) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= L.n) return;
    const double acc = spread_acc(k, L, M);
    const int c = L.cell[k];
    const int X = c % nx;
    const int t = c / nx;
    const int Y = t % ny, Z = t / ny;
    const double r = split_resid(g, c0, c1, X, Y, Z, nx, ny, nz, alpha, s) + scale * acc;
    const size_t j = ((size_t)Z * ny + Y) * (nx >> 1) + (X >> 1);
    if ((X + Y + Z) & 1) {
        f1[j] = (T)r;
    } else {
        f0[j] = (T)r;
        if (u0) u0[j] = (T)((T)r * (T)inv_diag);
    }
}

template <typename T>
void launch_resid_spread_enter(hipStream_t st, const SpreadLists& L, const SpreadMult& M, const double* g,
                               const T* c0, const T* c1, double scale, T* f0, T* f1, T* u0, int nx, int ny, int nz,
                               double alpha, double s, double inv_diag) {
    if (L.n <= 0) return;
    hipLaunchKernelGGL(k_resid_spread_enter<T>, dim3(nblocks(L.n)), dim3(kBlock), 0, st, L, M, g, c0, c1, scale, f0,
                       f1, u0, nx, ny, nz, alpha, s, inv_diag);
}
template void launch_resid_spread_enter<float>(hipStream_t, const SpreadLists&, const SpreadMult&, const double*,
                                               const float*, const float*, double, float*, float*, float*, int, int,
                                               int, double, double, double);
template void launch_resid_spread_enter<double>(hipStream_t, const SpreadLists&, const SpreadMult&, const double*,
                                                const double*, const double*, double, double*, double*, double*, int,
                                                int, int, double, double, double);

template <typename T>
__global__ void k_zero(T* __restrict__ p, size_t n) {
    const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = (T)0;
}

template <typename T>
void launch_zero(hipStream_t st, T* p, size_t n) {
    if (n == 0) return;
    hipLaunchKernelGGL(k_zero<T>, dim3(nblocks(n)), dim3(kBlock), 0, st, p, n);
}
template void launch_zero<float>(hipStream_t, float*, size_t);
template void launch_zero<double>(hipStream_t, double*, size_t);

// b0 = a0, b1 = a1 (two arrays of n elements each)
template <typename T>
__global__ void __launch_bounds__(kBlock) k_copy2(const T* __restrict__ a0, const T* __restrict__ a1,
                                                  T* __restrict__ b0, T* __restrict__ b1, size_t n) {
    const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    b0[i] = a0[i];
    b1[i] = a1[i];
}

template <typename T>
void launch_copy2(hipStream_t st, const T* a0, const T* a1, T* b0, T* b1, size_t n) {
    if (n == 0) return;
    hipLaunchKernelGGL(k_copy2<T>, dim3(nblocks(n)), dim3(kBlock), 0, st, a0, a1, b0, b1, n);
}
template void launch_copy2<float>(hipStream_t, const float*, const float*, float*, float*, size_t);
template void launch_copy2<double>(hipStream_t, const double*, const double*, double*, double*, size_t);

// ---------------------------------------------------------------------------
// N-vector kernels: one work-group of kFinBlock threads, fixed reduction order.

__global__ void __launch_bounds__(kFinBlock) k_nvec_project(double* v, int N) {
    constexpr int R = 12;  // values held per thread when N <= R * blockDim.x
    const int bd = (int)blockDim.x;
    if (N <= R * bd) {
        // every load issued before the first use: one memory latency, not N / blockDim.x
        double r[R];
#pragma unroll
        for (int c = 0; c < R; ++c) {
            const int i = threadIdx.x + c * bd;
            r[c] = i < N ? v[i] : 0.0;
        }
        double s = 0.0;
#pragma unroll
        for (int c = 0; c < R; ++c) s += r[c];
        const double m = wg_sum(s) / (double)N;
#pragma unroll
        for (int c = 0; c < R; ++c) {
            const int i = threadIdx.x + c * bd;
            if (i < N) v[i] = r[c] - m;
        }
        return;
    }
    double s = 0.0;
    for (int i = threadIdx.x; i < N; i += bd) s += v[i];
    const double m = wg_sum(s) / (double)N;
    for (int i = threadIdx.x; i < N; i += bd) v[i] -= m;
}

void launch_nvec_project(hipStream_t st, double* v, int N) {
    hipLaunchKernelGGL(k_nvec_project, dim3(1), dim3(kFinBlock), 0, st, v, N);
}

__global__ void k_nvec_copy_scale(const double* x, double* y, int N, double a, double shift) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < N) y[i] = (x ? a * x[i] : 0.0) + shift;
}

void launch_nvec_copy_scale(hipStream_t st, const double* x, double* y, int N, double a, double shift) {
    hipLaunchKernelGGL(k_nvec_copy_scale, dim3(nblocks(N)), dim3(kBlock), 0, st, x, y, N, a, shift);
}

__global__ void __launch_bounds__(kFinBlock) k_nvec_sums(const double* a, const double* b, int N, double* out) {
    double s0 = 0.0, s1 = 0.0, s2 = 0.0;
    for (int i = threadIdx.x; i < N; i += blockDim.x) {
        s0 += a[i];
        s1 += a[i] * a[i];
        if (b) s2 += a[i] * b[i];
    }
    s0 = wg_sum(s0);
    s1 = wg_sum(s1);
    s2 = wg_sum(s2);
    if (threadIdx.x == 0) {
        out[0] = s0;
        out[1] = s1;
        out[2] = s2;
    }
}

void launch_nvec_sums(hipStream_t st, const double* a, const double* b, int N, double* out) {
    hipLaunchKernelGGL(k_nvec_sums, dim3(1), dim3(kFinBlock), 0, st, a, b, N, out);
}

// GMRES cycle start: r = b - w (or b), beta = |r|, V_0 = r / beta, g = beta e_1.
// v_0 = r / |r| with r = b - w (has_w) or b, its mean removed first with project; g_0 = |r|.
__global__ void __launch_bounds__(kFinBlock) k_gmres_start(const double* b, const double* w, int has_w, double* V,
                                                           double* gvec, int N, GmresScalars* gs, int project) {
    double s = 0.0;
    for (int i = threadIdx.x; i < N; i += blockDim.x) {
        const double r = has_w ? b[i] - w[i] : b[i];
        V[i] = r;
        s += project ? r : r * r;
    }
    if (project) {
        const double mean = wg_sum(s) / (double)N;
        s = 0.0;
        for (int i = threadIdx.x; i < N; i += blockDim.x) {
            const double r = V[i] - mean;
            V[i] = r;
            s += r * r;
        }
    }
    const double beta = sqrt(wg_sum(s));
    const double inv = beta > 0.0 ? 1.0 / beta : 0.0;
    for (int i = threadIdx.x; i < N; i += blockDim.x) V[i] *= inv;
    if (threadIdx.x == 0) {
        gvec[0] = beta;
        gs->beta = beta;
        gs->res = beta;
        gs->k = 0;
        gs->status = (beta == beta) ? 0 : 1;
    }
}

void launch_gmres_start(hipStream_t st, const double* b, const double* w, int has_w, double* V, double* g, int N,
                        GmresScalars* gs, int project) {
    hipLaunchKernelGGL(k_gmres_start, dim3(1), dim3(kFinBlock), 0, st, b, w, has_w, V, g, N, gs, project);
}

// Arnoldi step k with modified Gram-Schmidt: V_{k+1} holds G v_k on entry
// (with project, its mean is removed first, as k_nvec_project does).
// H is (m+1) x m row-major; Givens rotations (cs, sn) update g.
// Elements of an N-vector a work-group thread keeps in registers during the
// modified Gram-Schmidt sweep (N <= kArnoldiRegs * kFinBlock).
constexpr int kArnoldiRegs = 12;

__global__ void __launch_bounds__(kFinBlock) k_gmres_arnoldi(double* V, double* H, double* cs, double* sn,
                                                             double* gvec, int N, int k, int m, GmresScalars* gs,
                                                             int project) {
    double* w = V + (size_t)(k + 1) * N;
    double hk1;
    if (N <= kArnoldiRegs * (int)blockDim.x) {
        // w stays in registers (the same sums, in the same order, as the
        // streaming form below)
        double wr[kArnoldiRegs];
#pragma unroll
        for (int c = 0; c < kArnoldiRegs; ++c) {
            const int i = threadIdx.x + c * blockDim.x;
            wr[c] = i < N ? w[i] : 0.0;
        }
        if (project) {
            double s = 0.0;
#pragma unroll
            for (int c = 0; c < kArnoldiRegs; ++c) s += wr[c];
            const double mean = wg_sum(s) / (double)N;
#pragma unroll
            for (int c = 0; c < kArnoldiRegs; ++c)
                if ((int)(threadIdx.x + c * blockDim.x) < N) wr[c] -= mean;
        }
        for (int j = 0; j <= k; ++j) {
            const double* vj = V + (size_t)j * N;
            double s = 0.0;
#pragma unroll
            for (int c = 0; c < kArnoldiRegs; ++c) {
                const int i = threadIdx.x + c * blockDim.x;
                if (i < N) s += wr[c] * vj[i];
            }
            const double hj = wg_sum(s);
#pragma unroll
            for (int c = 0; c < kArnoldiRegs; ++c) {
                const int i = threadIdx.x + c * blockDim.x;
                if (i < N) wr[c] -= hj * vj[i];  // v_j again from cache
            }
            if (threadIdx.x == 0) H[j * m + k] = hj;
        }
        double s = 0.0;
#pragma unroll
        for (int c = 0; c < kArnoldiRegs; ++c)
            if ((int)(threadIdx.x + c * blockDim.x) < N) s += wr[c] * wr[c];
        hk1 = sqrt(wg_sum(s));
        const double inv = hk1 > 0.0 ? 1.0 / hk1 : 0.0;
#pragma unroll
        for (int c = 0; c < kArnoldiRegs; ++c) {
            const int i = threadIdx.x + c * blockDim.x;
            if (i < N) w[i] = wr[c] * inv;
        }
    } else {
        if (project) {
            double s = 0.0;
            for (int i = threadIdx.x; i < N; i += blockDim.x) s += w[i];
            const double mean = wg_sum(s) / (double)N;
            for (int i = threadIdx.x; i < N; i += blockDim.x) w[i] -= mean;
        }
        for (int j = 0; j <= k; ++j) {
            const double* vj = V + (size_t)j * N;
            double s = 0.0;
            for (int i = threadIdx.x; i < N; i += blockDim.x) s += w[i] * vj[i];
            const double hj = wg_sum(s);
            for (int i = threadIdx.x; i < N; i += blockDim.x) w[i] -= hj * vj[i];
            if (threadIdx.x == 0) H[j * m + k] = hj;
        }
        double s = 0.0;
        for (int i = threadIdx.x; i < N; i += blockDim.x) s += w[i] * w[i];
        hk1 = sqrt(wg_sum(s));
        const double inv = hk1 > 0.0 ? 1.0 / hk1 : 0.0;
        for (int i = threadIdx.x; i < N; i += blockDim.x) w[i] *= inv;
    }
    if (threadIdx.x == 0) {
        H[(k + 1) * m + k] = hk1;
        for (int j = 0; j < k; ++j) {
            const double a = H[j * m + k], b = H[(j + 1) * m + k];
            H[j * m + k] = cs[j] * a + sn[j] * b;
            H[(j + 1) * m + k] = -sn[j] * a + cs[j] * b;
        }
        const double a = H[k * m + k], b = H[(k + 1) * m + k];
        const double den = sqrt(a * a + b * b);
        cs[k] = den == 0.0 ? 1.0 : a / den;
        sn[k] = den == 0.0 ? 0.0 : b / den;
        H[k * m + k] = den;
        H[(k + 1) * m + k] = 0.0;
        gvec[k + 1] = -sn[k] * gvec[k];
        gvec[k] = cs[k] * gvec[k];
        gs->res = fabs(gvec[k + 1]);
        gs->hk1 = hk1;
        gs->k = k + 1;
        if (!(den == den) || !(hk1 == hk1)) gs->status = 1;
    }
}

void launch_gmres_arnoldi(hipStream_t st, double* V, double* H, double* cs, double* sn, double* g, int N, int k,
                          int m, GmresScalars* gs, int project) {
    hipLaunchKernelGGL(k_gmres_arnoldi, dim3(1), dim3(kFinBlock), 0, st, V, H, cs, sn, g, N, k, m, gs, project);
}

// x += V y with H y = g (upper-triangular k x k), y solved by thread 0.
__global__ void __launch_bounds__(kFinBlock) k_gmres_update(const double* V, const double* H, const double* gvec,
                                                            double* y, double* x, int N, int k, int m) {
    if (threadIdx.x == 0) {
        for (int i = k - 1; i >= 0; --i) {
            double s = gvec[i];
            for (int j = i + 1; j < k; ++j) s -= H[i * m + j] * y[j];
            const double d = H[i * m + i];
            y[i] = d != 0.0 ? s / d : 0.0;
        }
    }
    __syncthreads();
    for (int i = threadIdx.x; i < N; i += blockDim.x) {
        double acc = x[i];
        for (int j = 0; j < k; ++j) acc += y[j] * V[(size_t)j * N + i];
        x[i] = acc;
    }
}

void launch_gmres_update(hipStream_t st, const double* V, const double* H, const double* g, double* y, double* x,
                         int N, int k, int m) {
    hipLaunchKernelGGL(k_gmres_update, dim3(1), dim3(kFinBlock), 0, st, V, H, g, y, x, N, k, m);
}

}  // namespace brd
