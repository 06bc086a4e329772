// Natural-layout FP64 grid kernels and the one-work-group finalize kernels.
//
// Operators (arXiv:1306.3159 Sec. III.A-III.B): A = alpha I - D L with L the
// periodic 7-point Laplacian; the CG vector updates of the multigrid-
// preconditioned Krylov solves of Sec. III.E.
#include "launch.hpp"

#include <cmath>

namespace brd {

// y = alpha x - s (sum of 6 neighbours - 6 x), s = D / h^2. BOX: a box with
// homogeneous faces, where the neighbour beyond a face is the ghost -x.
template <bool BOX>
__device__ __forceinline__ double stencil_A(const double* __restrict__ x, int X, int Y, int Z, int nx, int ny, int nz,
                                            double alpha, double s, size_t idx, double* center) {
    const long long sxy = (long long)nx * ny;
    const long long i = (long long)idx;
    const double c = x[i];
    double xm, xp, ym, yp, zm, zp;
    if (BOX) {
        xm = X > 0 ? x[i - 1] : -c;
        xp = X + 1 < nx ? x[i + 1] : -c;
        ym = Y > 0 ? x[i - nx] : -c;
        yp = Y + 1 < ny ? x[i + nx] : -c;
        zm = Z > 0 ? x[i - sxy] : -c;
        zp = Z + 1 < nz ? x[i + sxy] : -c;
    } else {
        xm = x[i - X + wrapi(X - 1, nx)];
        xp = x[i - X + wrapi(X + 1, nx)];
        ym = x[i + (long long)(wrapi(Y - 1, ny) - Y) * nx];
        yp = x[i + (long long)(wrapi(Y + 1, ny) - Y) * nx];
        zm = x[i + (long long)(wrapi(Z - 1, nz) - Z) * sxy];
        zp = x[i + (long long)(wrapi(Z + 1, nz) - Z) * sxy];
    }
    *center = c;
    return alpha * c - s * ((xm + xp) + (ym + yp) + (zm + zp) - 6.0 * c);
}

template <bool BOX>
__global__ void __launch_bounds__(kBlock) k_applyA(const double* __restrict__ p, double* __restrict__ q,
                                                   double alpha, double s, int nx, int ny, int nz, unsigned ncell,
                                                   double* part, const Scalars* sc) {
    if (sc && sc->done) return;
    unsigned lo, hi;
    chunk_of(xcd_block(blockIdx.x, gridDim.x), gridDim.x, ncell, &lo, &hi);
    double v[2] = {0.0, 0.0};
    for (unsigned idx = lo + threadIdx.x; idx < hi; idx += blockDim.x) {
        const int X = idx % nx;
        const unsigned t = idx / nx;
        const int Y = t % ny, Z = t / ny;
        double c;
        const double y = stencil_A<BOX>(p, X, Y, Z, nx, ny, nz, alpha, s, idx, &c);
        q[idx] = y;
        v[0] += c * y;
        v[1] += y;
    }
    if (part) block_partials<2>(v, part, gridDim.x, blockIdx.x);
}

void launch_applyA(hipStream_t st, const double* p, double* q, double alpha, double s, int nx, int ny, int nz,
                   double* part, const Scalars* sc, unsigned* np) {
    const unsigned n = (unsigned)nx * ny * nz;
    const unsigned nb = part ? red_blocks(n) : nblocks(n);
    hipLaunchKernelGGL(k_applyA<false>, dim3(nb), dim3(kBlock), 0, st, p, q, alpha, s, nx, ny, nz, n, part, sc);
    if (np) *np = nb;
}

typedef double double2_t __attribute__((ext_vector_type(2)));

// Two cells per thread (x even, x + 1) with 16-byte loads: q = alpha p - D L p,
// partials (p.q, sum q). Same arithmetic and summation order as stencil_A.
template <bool BOX>
__device__ __forceinline__ void applyA2_body(const double* __restrict__ p, double* __restrict__ q, double alpha,
                                             double s, int nx, int ny, int nz, unsigned npair, double* part, Blk blk,
                                             const double* __restrict__ base = nullptr) {
    unsigned lo, hi;
    chunk_of(xcd_block(blk.b, blk.nb), blk.nb, npair, &lo, &hi);
    double v[2] = {0.0, 0.0};
    const int hx = nx >> 1;
    const long long sxy = (long long)nx * ny;
    // kU pairs per pass: every load of the pass is issued before any of its pairs is
    // computed (a chunk of several pairs per thread then keeps kU x 7 loads in flight);
    // pairs are computed and summed in the chunk's order, as one at a time would be
    constexpr int kU = 4;
    const unsigned bd = blockDim.x;
    for (unsigned k0 = lo + threadIdx.x; k0 < hi; k0 += kU * bd) {
        long long i[kU];
        int X[kU];
        double2_t c[kU], ym[kU], yp[kU], zm[kU], zp[kU], b[kU];
        double xl[kU], xr[kU];
#pragma unroll
        for (int u = 0; u < kU; ++u) {
            const unsigned k = k0 + u * bd;
            if (k >= hi) continue;
            X[u] = 2 * (int)(k % hx);
            const unsigned t = k / hx;
            const int Y = t % ny, Z = t / ny;
            i[u] = ((long long)Z * ny + Y) * nx + X[u];
            c[u] = *reinterpret_cast<const double2_t*>(p + i[u]);
            if (BOX) {
                xl[u] = X[u] > 0 ? p[i[u] - 1] : -c[u][0];
                xr[u] = X[u] + 2 < nx ? p[i[u] + 2] : -c[u][1];
                ym[u] = Y > 0 ? *reinterpret_cast<const double2_t*>(p + i[u] - nx) : -c[u];
                yp[u] = Y + 1 < ny ? *reinterpret_cast<const double2_t*>(p + i[u] + nx) : -c[u];
                zm[u] = Z > 0 ? *reinterpret_cast<const double2_t*>(p + i[u] - sxy) : -c[u];
                zp[u] = Z + 1 < nz ? *reinterpret_cast<const double2_t*>(p + i[u] + sxy) : -c[u];
            } else {
                xl[u] = p[i[u] - X[u] + (X[u] == 0 ? nx - 1 : X[u] - 1)];
                xr[u] = p[i[u] - X[u] + (X[u] + 2 == nx ? 0 : X[u] + 2)];
                ym[u] = *reinterpret_cast<const double2_t*>(p + i[u] + (long long)(wrapi(Y - 1, ny) - Y) * nx);
                yp[u] = *reinterpret_cast<const double2_t*>(p + i[u] + (long long)(wrapi(Y + 1, ny) - Y) * nx);
                zm[u] = *reinterpret_cast<const double2_t*>(p + i[u] + (long long)(wrapi(Z - 1, nz) - Z) * sxy);
                zp[u] = *reinterpret_cast<const double2_t*>(p + i[u] + (long long)(wrapi(Z + 1, nz) - Z) * sxy);
            }
            if (base) b[u] = *reinterpret_cast<const double2_t*>(base + i[u]);
        }
#pragma unroll
        for (int u = 0; u < kU; ++u) {
            if (k0 + u * bd >= hi) continue;
            double2_t y;
            y[0] = alpha * c[u][0] - s * ((xl[u] + c[u][1]) + (ym[u][0] + yp[u][0]) + (zm[u][0] + zp[u][0]) -
                                          6.0 * c[u][0]);
            y[1] = alpha * c[u][1] - s * ((c[u][0] + xr[u]) + (ym[u][1] + yp[u][1]) + (zm[u][1] + zp[u][1]) -
                                          6.0 * c[u][1]);
            if (base) {  // residual form q = base - A p
                y[0] = b[u][0] - y[0];
                y[1] = b[u][1] - y[1];
            }
            *reinterpret_cast<double2_t*>(q + i[u]) = y;
            v[0] += c[u][0] * y[0] + c[u][1] * y[1];
            v[1] += y[0] + y[1];
        }
    }
    if (part) block_partials<2>(v, part, blk.nb, blk.b);
}

template <bool BOX>
__global__ void __launch_bounds__(kBlock) k_applyA2(const double* __restrict__ p, double* __restrict__ q,
                                                    double alpha, double s, int nx, int ny, int nz, unsigned npair,
                                                    double* part, const Scalars* sc) {
    if (sc && sc->done) return;
    applyA2_body<BOX>(p, q, alpha, s, nx, ny, nz, npair, part, Blk{blockIdx.x, gridDim.x});
}

// q = base - (alpha p - D L p), two cells per thread (no partials)
template <bool BOX>
__global__ void __launch_bounds__(kBlock) k_residA2(const double* __restrict__ base, const double* __restrict__ p,
                                                    double* __restrict__ q, double alpha, double s, int nx, int ny,
                                                    int nz, unsigned npair) {
    applyA2_body<BOX>(p, q, alpha, s, nx, ny, nz, npair, nullptr, Blk{blockIdx.x, gridDim.x}, base);
}

__global__ void __launch_bounds__(kBlock) kb_applyA2(const InstDev* inst, const int* gate, const BatchTab* tab) {
    const BatchEntry* ent = tab_entries(tab);
    for (unsigned g = blockIdx.x; g < tab->total; g += gridDim.x) {
        Blk blk;
        const InstDev* I = batch_slot(inst, gate, ent, tab->n, g, blk);
        if (!I) continue;
        applyA2_body<false>(I->p, I->q, I->alpha, I->ls[0], I->nx, I->ny, I->nz, (unsigned)(I->nx / 2) * I->ny * I->nz,
                     I->part, blk);
        __syncthreads();  // partial-sum scratch is reused by the next virtual block
    }
}

void launch_applyA2(hipStream_t st, const double* p, double* q, double alpha, double s, int nx, int ny, int nz,
                    double* part, const Scalars* sc, unsigned* np, bool box) {
    const unsigned npair = (unsigned)(nx / 2) * ny * nz;
    const unsigned nb = red_blocks(npair);
    hipLaunchKernelGGL(box ? k_applyA2<true> : k_applyA2<false>, dim3(nb), dim3(kBlock), 0, st, p, q, alpha, s, nx,
                       ny, nz, npair, part, sc);
    *np = nb;
}

// p = z + shift + beta p, two cells per thread (z from the split level-0 arrays)
template <typename T>
__device__ __forceinline__ void dir2_body(const T* __restrict__ z0, const T* __restrict__ z1, double* __restrict__ p,
                                          int nx, int ny, unsigned npair, double beta, double shift, Blk blk) {
    const unsigned k = xcd_block(blk.b, blk.nb) * blockDim.x + threadIdx.x;
    if (k >= npair) return;
    const int hx = nx >> 1;
    const unsigned t = k / hx;
    const int Y = t % ny, Z = t / ny;
    const int par = (Y + Z) & 1;  // colour of the even cell
    const double za = (double)(par ? z1[k] : z0[k]) + shift;
    const double zb = (double)(par ? z0[k] : z1[k]) + shift;
    double2_t* pp = reinterpret_cast<double2_t*>(p) + k;
    double2_t v;
    if (beta == 0.0) {
        v[0] = za;
        v[1] = zb;
    } else {
        const double2_t o = *pp;
        v[0] = za + beta * o[0];
        v[1] = zb + beta * o[1];
    }
    *pp = v;
}

template <typename T>
__global__ void __launch_bounds__(kBlock) k_dir2(const T* __restrict__ z0, const T* __restrict__ z1,
                                                 double* __restrict__ p, int nx, int ny, unsigned npair,
                                                 const Scalars* sc) {
    if (sc->done) return;
    dir2_body<T>(z0, z1, p, nx, ny, npair, sc->beta, sc->shift, Blk{blockIdx.x, gridDim.x});
}

template <typename T>
__global__ void __launch_bounds__(kBlock) kb_dir2(const InstDev* inst, const int* gate, const BatchTab* tab) {
    const BatchEntry* ent = tab_entries(tab);
    for (unsigned g = blockIdx.x; g < tab->total; g += gridDim.x) {
        Blk blk;
        const InstDev* I = batch_slot(inst, gate, ent, tab->n, g, blk);
        if (!I) continue;
        dir2_body<T>(static_cast<const T*>(I->lv[0][0]), static_cast<const T*>(I->lv[0][1]), I->p, I->nx, I->ny,
                     (unsigned)(I->nx / 2) * I->ny * I->nz, I->sc->beta, I->sc->shift, blk);
    }
}

template <typename T>
void launch_dir2(hipStream_t st, const T* z0, const T* z1, double* p, int nx, int ny, int nz, const Scalars* sc) {
    const unsigned npair = (unsigned)(nx / 2) * ny * nz;
    hipLaunchKernelGGL(k_dir2<T>, dim3(nblocks(npair)), dim3(kBlock), 0, st, z0, z1, p, nx, ny, npair, sc);
}
template void launch_dir2<float>(hipStream_t, const float*, const float*, double*, int, int, int, const Scalars*);
template void launch_dir2<double>(hipStream_t, const double*, const double*, double*, int, int, int, const Scalars*);

// x += alpha p ; r -= alpha q with partials (r.r, sum r), and the V-cycle
// entry for the new r in the same pass: f = r - mean (the mean predicted from
// sum r and sum q) into the split level-0 arrays, and the first red
// half-sweep from a zero guess, u_red = f_red / diag (as k_enter computes it).
// BOX: the diagonal of a box with fixed faces, per red cell from its face count.
template <typename T, bool BOX = false>
__device__ __forceinline__ void update2_enter_body(double* __restrict__ x, double* __restrict__ r,
                                                   const double* __restrict__ p, const double* __restrict__ q,
                                                   T* __restrict__ f0, T* __restrict__ f1, T* __restrict__ u0, int nx,
                                                   int ny, unsigned npair, double inv_diag, double a, double m,
                                                   bool fresh, double* part, Blk blk, int nz = 0,
                                                   BoxCoef binv = BoxCoef{}) {
    unsigned lo, hi;
    chunk_of(xcd_block(blk.b, blk.nb), blk.nb, npair, &lo, &hi);
    double v[2] = {0.0, 0.0};
    const int hx = nx >> 1;
    for (unsigned k = lo + threadIdx.x; k < hi; k += blockDim.x) {
        // fresh: x starts at zero and is not read (the first step of a zero-start run)
        double2_t xv = fresh ? double2_t{0.0, 0.0} : reinterpret_cast<double2_t*>(x)[k];
        double2_t rv = reinterpret_cast<double2_t*>(r)[k];
        const double2_t pv = reinterpret_cast<const double2_t*>(p)[k];
        const double2_t qv = reinterpret_cast<const double2_t*>(q)[k];
        xv[0] += a * pv[0];
        xv[1] += a * pv[1];
        rv[0] -= a * qv[0];
        rv[1] -= a * qv[1];
        reinterpret_cast<double2_t*>(x)[k] = xv;
        reinterpret_cast<double2_t*>(r)[k] = rv;
        v[0] += rv[0] * rv[0] + rv[1] * rv[1];
        v[1] += rv[0] + rv[1];
        const unsigned t = k / hx;
        const int par = ((int)(t % ny) + (int)(t / ny)) & 1;  // colour of the even cell
        const double fa = rv[0] - m, fb = rv[1] - m;
        const double fr = par ? fb : fa, fk = par ? fa : fb;
        f0[k] = (T)fr;
        f1[k] = (T)fk;
        if (BOX) {
            const int xr = 2 * (int)(k % hx) + par;  // the red cell of the pair
            u0[k] = (T)((T)fr * (T)binv.v[box_faces(xr, (int)(t % ny), (int)(t / ny), nx, ny, nz)]);
        } else {
            u0[k] = (T)((T)fr * (T)inv_diag);
        }
    }
    block_partials<2>(v, part, blk.nb, blk.b);
}

template <typename T>
__global__ void __launch_bounds__(kBlock) k_update2_enter(double* __restrict__ x, double* __restrict__ r,
                                                          const double* __restrict__ p, const double* __restrict__ q,
                                                          T* __restrict__ f0, T* __restrict__ f1, T* __restrict__ u0,
                                                          int nx, int ny, unsigned npair, double inv_diag,
                                                          double* part, const Scalars* sc) {
    if (sc->done) return;
    update2_enter_body<T>(x, r, p, q, f0, f1, u0, nx, ny, npair, inv_diag, sc->alpha, sc->mean_next,
                          sc->xzero && sc->iters == 0, part, Blk{blockIdx.x, gridDim.x});
}

template <typename T>
__global__ void __launch_bounds__(kBlock) k_update2_enter_box(double* __restrict__ x, double* __restrict__ r,
                                                              const double* __restrict__ p,
                                                              const double* __restrict__ q, T* __restrict__ f0,
                                                              T* __restrict__ f1, T* __restrict__ u0, int nx, int ny,
                                                              int nz, unsigned npair, BoxCoef binv, double* part,
                                                              const Scalars* sc) {
    if (sc->done) return;
    update2_enter_body<T, true>(x, r, p, q, f0, f1, u0, nx, ny, npair, 0.0, sc->alpha, sc->mean_next,
                                sc->xzero && sc->iters == 0, part, Blk{blockIdx.x, gridDim.x}, nz, binv);
}

template <typename T>
__global__ void __launch_bounds__(kBlock) kb_update2_enter(const InstDev* inst, const int* gate, const BatchTab* tab) {
    const BatchEntry* ent = tab_entries(tab);
    for (unsigned g = blockIdx.x; g < tab->total; g += gridDim.x) {
        Blk blk;
        const InstDev* I = batch_slot(inst, gate, ent, tab->n, g, blk);
        if (!I) continue;
        update2_enter_body<T>(I->x, I->r, I->p, I->q, static_cast<T*>(I->lv[0][2]), static_cast<T*>(I->lv[0][3]),
                              static_cast<T*>(I->lv[0][0]), I->nx, I->ny, (unsigned)(I->nx / 2) * I->ny * I->nz,
                              1.0 / I->ldiag[0], I->sc->alpha, I->sc->mean_next,
                              I->sc->xzero && I->sc->iters == 0, I->part, blk);
        __syncthreads();  // partial-sum scratch is reused by the next virtual block
    }
}

template <typename T>
void launch_update2_enter(hipStream_t st, double* x, double* r, const double* p, const double* q, T* f0, T* f1, T* u0,
                          int nx, int ny, int nz, double inv_diag, double* part, const Scalars* sc, unsigned* np,
                          const BoxCoef* box_inv) {
    const unsigned npair = (unsigned)(nx / 2) * ny * nz;
    const unsigned nb = red_blocks(npair);
    if (box_inv)
        hipLaunchKernelGGL(k_update2_enter_box<T>, dim3(nb), dim3(kBlock), 0, st, x, r, p, q, f0, f1, u0, nx, ny, nz,
                           npair, *box_inv, part, sc);
    else
        hipLaunchKernelGGL(k_update2_enter<T>, dim3(nb), dim3(kBlock), 0, st, x, r, p, q, f0, f1, u0, nx, ny, npair,
                           inv_diag, part, sc);
    *np = nb;
}
template void launch_update2_enter<float>(hipStream_t, double*, double*, const double*, const double*, float*, float*,
                                          float*, int, int, int, double, double*, const Scalars*, unsigned*,
                                          const BoxCoef*);
template void launch_update2_enter<double>(hipStream_t, double*, double*, const double*, const double*, double*,
                                           double*, double*, int, int, int, double, double*, const Scalars*,
                                           unsigned*, const BoxCoef*);

// partials (sum z, z.r, z.q), two cells per thread
template <typename T>
__global__ void __launch_bounds__(kBlock) k_zdots2(const T* __restrict__ z0, const T* __restrict__ z1,
                                                   const double* __restrict__ r, const double* __restrict__ q,
                                                   int nx, int ny, unsigned npair, double* part, const Scalars* sc) {
    if (sc->done) return;
    unsigned lo, hi;
    chunk_of(xcd_block(blockIdx.x, gridDim.x), gridDim.x, npair, &lo, &hi);
    double v[3] = {0.0, 0.0, 0.0};
    const int hx = nx >> 1;
    for (unsigned k = lo + threadIdx.x; k < hi; k += blockDim.x) {
        const unsigned t = k / hx;
        const int par = ((int)(t % ny) + (int)(t / ny)) & 1;
        const double za = (double)(par ? z1[k] : z0[k]);
        const double zb = (double)(par ? z0[k] : z1[k]);
        const double2_t rv = reinterpret_cast<const double2_t*>(r)[k];
        const double2_t qv = reinterpret_cast<const double2_t*>(q)[k];
        v[0] += za + zb;
        v[1] += za * rv[0] + zb * rv[1];
        v[2] += za * qv[0] + zb * qv[1];
    }
    block_partials<3>(v, part, gridDim.x, blockIdx.x);
}

template <typename T>
void launch_zdots2(hipStream_t st, const T* z0, const T* z1, const double* r, const double* q, int nx, int ny, int nz,
                   double* part, const Scalars* sc, unsigned* np) {
    const unsigned npair = (unsigned)(nx / 2) * ny * nz;
    const unsigned nb = red_blocks(npair);
    hipLaunchKernelGGL(k_zdots2<T>, dim3(nb), dim3(kBlock), 0, st, z0, z1, r, q, nx, ny, npair, part, sc);
    *np = nb;
}
template void launch_zdots2<float>(hipStream_t, const float*, const float*, const double*, const double*, int, int,
                                   int, double*, const Scalars*, unsigned*);
template void launch_zdots2<double>(hipStream_t, const double*, const double*, const double*, const double*, int,
                                    int, int, double*, const Scalars*, unsigned*);

// pairs of cells per thread of the plain stencil launches (BLOB_RD_STENCIL_PAIRS, default 2:
// at 256^3 38 us warm and 71 us cold against 50 and 77 with one pair per thread)
unsigned stencil_pairs() {
    static const unsigned v = [] {
        const char* e = std::getenv("BLOB_RD_STENCIL_PAIRS");
        const int k = e ? std::atoi(e) : 2;
        return (unsigned)(k >= 1 && k <= 16 ? k : 2);
    }();
    return v;
}

void launch_applyA_plain(hipStream_t st, const double* x, double* y, double alpha, double s, int nx, int ny,
                         int nz, bool box) {
    const unsigned n = (unsigned)nx * ny * nz;
    if (nx % 2 == 0) {  // two cells per thread, the same arithmetic
        const unsigned npair = n / 2;
        hipLaunchKernelGGL(box ? k_applyA2<true> : k_applyA2<false>, dim3(nblocks(npair, kBlock * stencil_pairs())),
                           dim3(kBlock), 0, st, x, y, alpha, s, nx, ny, nz, npair, (double*)nullptr,
                           (const Scalars*)nullptr);
        return;
    }
    hipLaunchKernelGGL(box ? k_applyA<true> : k_applyA<false>, dim3(nblocks(n)), dim3(kBlock), 0, st, x, y, alpha,
                       s, nx, ny, nz, n, (double*)nullptr, (const Scalars*)nullptr);
}

void launch_residA_plain(hipStream_t st, const double* base, const double* x, double* q, double alpha, double s,
                         int nx, int ny, int nz, bool box) {
    const unsigned n = (unsigned)nx * ny * nz;
    if (nx % 2 == 0) {
        const unsigned npair = n / 2;
        hipLaunchKernelGGL(box ? k_residA2<true> : k_residA2<false>, dim3(nblocks(npair, kBlock * stencil_pairs())),
                           dim3(kBlock), 0, st, base, x, q, alpha, s, nx, ny, nz, npair);
        return;
    }
    launch_applyA_plain(st, x, q, alpha, s, nx, ny, nz, box);
    launch_axpby(st, q, base, n, -1.0, 1.0);
}

// r = g - (alpha x - D L x) or, with x == nullptr, r = g - q0 (q0 may be null: r = g).
__global__ void __launch_bounds__(kBlock) k_residual64(const double* __restrict__ g, const double* __restrict__ x,
                                                       const double* __restrict__ q0, double* __restrict__ r,
                                                       double alpha, double s, int nx, int ny, int nz,
                                                       unsigned ncell, double* part) {
    unsigned lo, hi;
    chunk_of(xcd_block(blockIdx.x, gridDim.x), gridDim.x, ncell, &lo, &hi);
    double v[3] = {0.0, 0.0, 0.0};
    for (unsigned idx = lo + threadIdx.x; idx < hi; idx += blockDim.x) {
        double ax = 0.0;
        if (x) {
            const int X = idx % nx;
            const unsigned t = idx / nx;
            double c;
            ax = stencil_A<false>(x, X, (int)(t % ny), (int)(t / ny), nx, ny, nz, alpha, s, idx, &c);
        } else if (q0) {
            ax = q0[idx];
        }
        const double gv = g[idx];
        const double rv = gv - ax;
        r[idx] = rv;
        v[0] += rv * rv;
        v[1] += rv;
        v[2] += gv * gv;
    }
    block_partials<3>(v, part, gridDim.x, blockIdx.x);
}

// The partials of launch_residual_from_q(g, null, r) when r already holds g:
// (g.g, sum g, g.g), same chunks and order.
__global__ void __launch_bounds__(kBlock) k_self_partials(const double* __restrict__ g, unsigned n, double* part) {
    unsigned lo, hi;
    chunk_of(xcd_block(blockIdx.x, gridDim.x), gridDim.x, n, &lo, &hi);
    double v[3] = {0.0, 0.0, 0.0};
    for (unsigned idx = lo + threadIdx.x; idx < hi; idx += blockDim.x) {
        const double gv = g[idx];
        const double rv = gv - 0.0;
        v[0] += rv * rv;
        v[1] += rv;
        v[2] += gv * gv;
    }
    block_partials<3>(v, part, gridDim.x, blockIdx.x);
}

void launch_self_partials(hipStream_t st, const double* g, size_t n, double* part, unsigned* np) {
    const unsigned nb = red_blocks(n);
    hipLaunchKernelGGL(k_self_partials, dim3(nb), dim3(kBlock), 0, st, g, (unsigned)n, part);
    *np = nb;
}

void launch_residual_from_q(hipStream_t st, const double* g, const double* q0, double* r, size_t n, double* part,
                            unsigned* np) {
    const unsigned nb = red_blocks(n);
    hipLaunchKernelGGL(k_residual64, dim3(nb), dim3(kBlock), 0, st, g, (const double*)nullptr, q0, r, 0.0, 0.0, 1,
                       1, 1, (unsigned)n, part);
    *np = nb;
}

// Split-layout value at natural (X, Y, Z) of level 0.

// out = scale * out + z (+ shift_scale * *shift_dev)   (z split -> natural)
template <typename T>
__global__ void __launch_bounds__(kBlock) k_split_to_nat(const T* __restrict__ z0, const T* __restrict__ z1,
                                                         double* __restrict__ out, int nx, int ny, unsigned ncell,
                                                         double scale, const double* __restrict__ shift_dev,
                                                         double shift_scale) {
    const unsigned idx = blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= ncell) return;
    const int X = idx % nx;
    const unsigned t = idx / nx;
    const double zv = split_at(z0, z1, X, (int)(t % ny), (int)(t / ny), nx >> 1, ny);
    double v = scale == 0.0 ? zv : scale * out[idx] + zv;
    if (shift_dev) v += shift_scale * shift_dev[0];
    out[idx] = v;
}

// Pair form: the element j of each colour array per thread, i.e. the natural cells
// x = 2i and 2i + 1 of a row (x = 2i has colour (y + z) & 1, x = 2i + 1 the other), which
// sit at 2j and 2j + 1 of the natural vector; each computed as in the one-cell form.
template <typename T>
__global__ void __launch_bounds__(kBlock) k_split_to_nat2(const T* __restrict__ z0, const T* __restrict__ z1,
                                                          double* __restrict__ out, int hx, int ny, unsigned nh,
                                                          double scale, const double* __restrict__ shift_dev,
                                                          double shift_scale) {
    typedef double D2 __attribute__((ext_vector_type(2)));
    const unsigned idx = blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= nh) return;
    const unsigned t = idx / hx;  // row z * ny + y
    const int p = ((int)(t % ny) + (int)(t / ny)) & 1;
    const double a = (double)z0[idx], b = (double)z1[idx];
    const double e0 = p ? b : a, e1 = p ? a : b;
    D2* o = reinterpret_cast<D2*>(out) + idx;
    double v0, v1;
    if (scale == 0.0) {
        v0 = e0;
        v1 = e1;
    } else {
        const D2 prev = *o;
        v0 = scale * prev[0] + e0;
        v1 = scale * prev[1] + e1;
    }
    if (shift_dev) {
        v0 += shift_scale * shift_dev[0];
        v1 += shift_scale * shift_dev[0];
    }
    *o = D2{v0, v1};
}

template <typename T>
void launch_split_to_nat(hipStream_t st, const T* z0, const T* z1, double* out, int nx, int ny, int nz,
                         double scale, const double* shift_dev, double shift_scale) {
    if (nx % 2 == 0) {
        const unsigned nh = (unsigned)(nx / 2) * ny * nz;
        hipLaunchKernelGGL(k_split_to_nat2<T>, dim3(nblocks(nh)), dim3(kBlock), 0, st, z0, z1, out, nx / 2, ny, nh,
                           scale, shift_dev, shift_scale);
        return;
    }
    const unsigned n = (unsigned)nx * ny * nz;
    hipLaunchKernelGGL(k_split_to_nat<T>, dim3(nblocks(n)), dim3(kBlock), 0, st, z0, z1, out, nx, ny, n, scale,
                       shift_dev, shift_scale);
}
template void launch_split_to_nat<float>(hipStream_t, const float*, const float*, double*, int, int, int, double,
                                         const double*, double);
template void launch_split_to_nat<double>(hipStream_t, const double*, const double*, double*, int, int, int, double,
                                          const double*, double);

// out = (b + z) + shift_scale * *shift_dev with b and z in the split layout (pair form, nx
// even): what k_split_to_nat2 with scale 1 writes when out holds the natural copy of b.
template <typename T>
__global__ void __launch_bounds__(kBlock) k_split_add_to_nat2(const T* __restrict__ b0, const T* __restrict__ b1,
                                                              const T* __restrict__ z0, const T* __restrict__ z1,
                                                              double* __restrict__ out, int hx, int ny, unsigned nh,
                                                              const double* __restrict__ shift_dev,
                                                              double shift_scale) {
    typedef double D2 __attribute__((ext_vector_type(2)));
    const unsigned idx = blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= nh) return;
    const unsigned t = idx / hx;  // row z * ny + y
    const int p = ((int)(t % ny) + (int)(t / ny)) & 1;
    const double a = (double)z0[idx], b = (double)z1[idx];
    const double ba = (double)b0[idx], bb = (double)b1[idx];
    double v0 = (p ? bb : ba) + (p ? b : a);
    double v1 = (p ? ba : bb) + (p ? a : b);
    if (shift_dev) {
        v0 += shift_scale * shift_dev[0];
        v1 += shift_scale * shift_dev[0];
    }
    reinterpret_cast<D2*>(out)[idx] = D2{v0, v1};
}

template <typename T>
void launch_split_add_to_nat(hipStream_t st, const T* b0, const T* b1, const T* z0, const T* z1, double* out, int nx,
                             int ny, int nz, const double* shift_dev, double shift_scale) {
    const unsigned nh = (unsigned)(nx / 2) * ny * nz;
    hipLaunchKernelGGL(k_split_add_to_nat2<T>, dim3(nblocks(nh)), dim3(kBlock), 0, st, b0, b1, z0, z1, out, nx / 2,
                       ny, nh, shift_dev, shift_scale);
}
template void launch_split_add_to_nat<float>(hipStream_t, const float*, const float*, const float*, const float*,
                                             double*, int, int, int, const double*, double);
template void launch_split_add_to_nat<double>(hipStream_t, const double*, const double*, const double*,
                                              const double*, double*, int, int, int, const double*, double);

__global__ void __launch_bounds__(kBlock) k_norm_partials(const double* __restrict__ v, unsigned n, double* part) {
    unsigned lo, hi;
    chunk_of(blockIdx.x, gridDim.x, n, &lo, &hi);
    double a[2] = {0.0, 0.0};
    for (unsigned idx = lo + threadIdx.x; idx < hi; idx += blockDim.x) {
        a[0] += v[idx];
        a[1] += v[idx] * v[idx];
    }
    block_partials<2>(a, part, gridDim.x, blockIdx.x);
}

void launch_norm_partials(hipStream_t st, const double* v, size_t n, double* part, unsigned* np) {
    const unsigned nb = red_blocks(n);
    hipLaunchKernelGGL(k_norm_partials, dim3(nb), dim3(kBlock), 0, st, v, (unsigned)n, part);
    *np = nb;
}

// Measurement probe: out = a + b over n16 16-byte vectors, the launch shape of the vector
// half-sweep (one vector per thread, XCD-mapped blocks): the bandwidth a plain streaming
// launch of the sweep's size reaches, the ceiling its roofline fraction is read against.
__global__ void __launch_bounds__(kBlock) k_stream_add(const float4* __restrict__ a, const float4* __restrict__ b,
                                                       float4* __restrict__ out, unsigned n16) {
    const unsigned idx = xcd_block(blockIdx.x, gridDim.x) * blockDim.x + threadIdx.x;
    if (idx >= n16) return;
    const float4 x = a[idx], y = b[idx];
    out[idx] = make_float4(x.x + y.x, x.y + y.y, x.z + y.z, x.w + y.w);
}
void launch_stream_add(hipStream_t st, const void* a, const void* b, void* out, size_t bytes) {
    const unsigned n16 = (unsigned)(bytes / 16);
    hipLaunchKernelGGL(k_stream_add, dim3(nblocks(n16)), dim3(kBlock), 0, st, (const float4*)a, (const float4*)b,
                       (float4*)out, n16);
}

__global__ void k_fill(double* v, unsigned n, double value) {
    const unsigned idx = blockIdx.x * blockDim.x + threadIdx.x;
    if (idx < n) v[idx] = value;
}
void launch_fill(hipStream_t st, double* v, size_t n, double value) {
    hipLaunchKernelGGL(k_fill, dim3(nblocks(n)), dim3(kBlock), 0, st, v, (unsigned)n, value);
}

__global__ void k_axpby(double* y, const double* x, unsigned n, double a, double b) {
    const unsigned idx = blockIdx.x * blockDim.x + threadIdx.x;
    if (idx < n) y[idx] = (a == 0.0 ? 0.0 : a * y[idx]) + b * x[idx];
}
void launch_axpby(hipStream_t st, double* y, const double* x, size_t n, double a, double b) {
    hipLaunchKernelGGL(k_axpby, dim3(nblocks(n)), dim3(kBlock), 0, st, y, x, (unsigned)n, a, b);
}

__global__ void k_add_shift(double* v, unsigned n, const double* shift, double sign) {
    const unsigned idx = blockIdx.x * blockDim.x + threadIdx.x;
    if (idx < n) v[idx] += sign * shift[0];
}
void launch_add_shift(hipStream_t st, double* v, size_t n, const double* shift_dev, double sign) {
    hipLaunchKernelGGL(k_add_shift, dim3(nblocks(n)), dim3(kBlock), 0, st, v, (unsigned)n, shift_dev, sign);
}

// ---------------------------------------------------------------------------
// Finalize: one work-group of kFinBlock threads reduces block partials in a
// fixed order and advances the CG scalars.
// ---------------------------------------------------------------------------
__device__ __forceinline__ double fin_sum(const double* __restrict__ p, unsigned n) {
    __shared__ double sh[kFinBlock / 64];
    double s = 0.0;
    for (unsigned i = threadIdx.x; i < n; i += blockDim.x) s += p[i];
    s = wave_sum(s);
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    __syncthreads();
    if (lane == 0) sh[wid] = s;
    __syncthreads();
    double t = 0.0;
    for (int w = 0; w < (int)(blockDim.x >> 6); ++w) t += sh[w];
    __syncthreads();
    return t;
}

__device__ __forceinline__ bool is_finite_d(double v) { return v == v && v - v == 0.0; }

__device__ __forceinline__ void fin_body(int kind, const double* __restrict__ part, unsigned np, Scalars* sc,
                                         const double* __restrict__ na, const double* __restrict__ nb, int nblob,
                                         double inv_h3) {
    if (kind == FIN_INIT) {
        const double rr = fin_sum(part, np);
        const double rs = fin_sum(part + np, np);
        const double gg = fin_sum(part + 2 * (size_t)np, np);
        if (threadIdx.x == 0) {
            // On entry tol2 holds rtol^2 and rr0 holds an absolute floor^2.
            const double t2 = fmax(sc->tol2 * gg, sc->rr0);
            sc->rr = rr;
            sc->rr0 = rr;
            sc->rsum = rs;
            sc->gg = gg;
            sc->tol2 = t2;
            sc->iters = 0;
            sc->beta = 0.0;
            sc->status = is_finite_d(rr) ? 0 : 1;
            sc->done = (rr <= t2 || !is_finite_d(rr)) ? 1 : 0;
            sc->mean_r = sc->project ? rs * sc->inv_ncell : 0.0;
        }
    } else if (kind == FIN_ALPHA) {
        double pq = fin_sum(part, np);
        double qs = fin_sum(part + np, np);
        if (na && nb) {
            // blob term of B: p.(S mu) = h^-3 (J p).mu, sum(S mu) = h^-3 sum(mu)
            double a = 0.0, c = 0.0;
            for (int i = threadIdx.x; i < nblob; i += blockDim.x) {
                a += na[i] * nb[i];
                c += nb[i];
            }
            __shared__ double sh2[2][kFinBlock / 64];
            a = wave_sum(a);
            c = wave_sum(c);
            if ((threadIdx.x & 63) == 0) {
                sh2[0][threadIdx.x >> 6] = a;
                sh2[1][threadIdx.x >> 6] = c;
            }
            __syncthreads();
            double ta = 0.0, tc = 0.0;
            for (int w = 0; w < (int)(blockDim.x >> 6); ++w) {
                ta += sh2[0][w];
                tc += sh2[1][w];
            }
            pq += inv_h3 * ta;
            qs += inv_h3 * tc;
        }
        if (threadIdx.x == 0) {
            sc->pq = pq;
            sc->qsum = qs;
            sc->mean_next = 0.0;
            if (!(pq > 0.0) || !is_finite_d(pq) || !is_finite_d(sc->rz)) {
                sc->status = 1;
                sc->done = 1;
                sc->alpha = 0.0;
            } else {
                sc->alpha = sc->rz / pq;
                // sum(r - alpha q) = sum r - alpha sum q: the mean the fused update removes
                if (sc->project) sc->mean_next = (sc->rsum - sc->alpha * qs) * sc->inv_ncell;
            }
        }
    } else if (kind == FIN_UPDATE) {
        const double rr = fin_sum(part, np);
        const double rs = fin_sum(part + np, np);
        if (threadIdx.x == 0) {
            sc->rr = rr;
            sc->rsum = rs;
            sc->iters += 1;
            sc->mean_r = sc->project ? rs * sc->inv_ncell : 0.0;
            if (!is_finite_d(rr)) {
                sc->status = 1;
                sc->done = 1;
            } else if (rr <= sc->tol2) {
                sc->done = 1;
            }
        }
    } else {  // FIN_BETA
        const double zs = fin_sum(part, np);
        const double zr = fin_sum(part + np, np);
        const double zq = fin_sum(part + 2 * (size_t)np, np);
        if (threadIdx.x == 0) {
            const double shift = sc->project ? (sc->rsum * sc->eBe_inv - zs * sc->inv_ncell) : 0.0;
            const double rz_new = zr + shift * sc->rsum;
            const double zq_full = zq + shift * sc->qsum;
            sc->shift = shift;
            if (sc->iters == 0) {
                sc->beta = 0.0;
            } else {
                sc->beta = -sc->alpha * zq_full / sc->rz;
            }
            sc->rz = rz_new;
            if (!is_finite_d(rz_new) || !is_finite_d(sc->beta)) {
                sc->status = 1;
                sc->done = 1;
            }
        }
    }
}

__global__ void __launch_bounds__(kFinBlock) k_fin(int kind, const double* __restrict__ part, unsigned np,
                                                   Scalars* sc, const double* __restrict__ na,
                                                   const double* __restrict__ nb, int nblob, double inv_h3) {
    if (kind != FIN_INIT && sc->done) return;
    fin_body(kind, part, np, sc, na, nb, nblob, inv_h3);
}

void launch_fin(hipStream_t st, int kind, const double* part, unsigned np, Scalars* sc, const double* na,
                const double* nb, int nblob, double inv_h3) {
    hipLaunchKernelGGL(k_fin, dim3(1), dim3(kFinBlock), 0, st, kind, part, np, sc, na, nb, nblob, inv_h3);
}

// One work-group per instance: FIN_ALPHA (with the blob sums of blob
// instances), FIN_UPDATE or FIN_BETA of every gated, unfinished instance.
__global__ void __launch_bounds__(kFinBlock) kb_fin(int kind, const InstDev* inst, const int* gate, int ninst) {
    const int i = blockIdx.x;
    if (i >= ninst || !gate[i]) return;
    const InstDev* I = inst + i;
    if (I->sc->done) return;
    const unsigned np = kind == FIN_ALPHA ? I->np_apply : kind == FIN_UPDATE ? I->np_update : I->np_dots;
    const bool blob = kind == FIN_ALPHA && I->blobs;
    fin_body(kind, I->part, np, I->sc, blob ? I->jx : nullptr, blob ? I->mu : nullptr, blob ? I->N : 0, I->inv_h3);
}

template <typename T>
void launchb_cg(hipStream_t st, int what, const InstDev* inst, const int* gate, const BatchTab* tab, unsigned grid,
                int ninst) {
    const dim3 g(grid), b(kBlock);
    switch (what) {
        case BCG_DIR: hipLaunchKernelGGL(kb_dir2<T>, g, b, 0, st, inst, gate, tab); break;
        case BCG_APPLY: hipLaunchKernelGGL(kb_applyA2, g, b, 0, st, inst, gate, tab); break;
        case BCG_UPDATE: hipLaunchKernelGGL(kb_update2_enter<T>, g, b, 0, st, inst, gate, tab); break;
        default:
            hipLaunchKernelGGL(kb_fin, dim3(ninst), dim3(kFinBlock), 0, st,
                               what == BCG_FIN_ALPHA ? FIN_ALPHA : what == BCG_FIN_UPDATE ? FIN_UPDATE : FIN_BETA,
                               inst, gate, ninst);
    }
}
template void launchb_cg<float>(hipStream_t, int, const InstDev*, const int*, const BatchTab*, unsigned, int);
template void launchb_cg<double>(hipStream_t, int, const InstDev*, const int*, const BatchTab*, unsigned, int);

__global__ void __launch_bounds__(kFinBlock) k_reduce_parts(const double* __restrict__ part, unsigned np, int k,
                                                            double* out) {
    for (int j = 0; j < k; ++j) {
        const double s = fin_sum(part + (size_t)j * np, np);
        if (threadIdx.x == 0) out[j] = s;
    }
}

void launch_reduce_parts(hipStream_t st, const double* part, unsigned np, int k, double* out) {
    hipLaunchKernelGGL(k_reduce_parts, dim3(1), dim3(kFinBlock), 0, st, part, np, k, out);
}

// ---------------------------------------------------------------------------
// Long vectors of the flexible GMRES on the block saddle system: a grid part of
// ncell values followed by N blob values, n = ncell + N doubles, each vector
// 16-byte aligned. Two values per thread (16-byte loads), one scalar tail.
// ---------------------------------------------------------------------------

// One modified Gram-Schmidt pass: w -= (*hprev) vprev when vprev is set, then
// partials of w.vnext (of w.w when vnext is null) into part[block].
__global__ void __launch_bounds__(kBlock) k_fg_mgs(double* __restrict__ w, const double* __restrict__ vprev,
                                                   const double* __restrict__ hprev, const double* __restrict__ vnext,
                                                   unsigned n, double* part) {
    const unsigned n2 = n >> 1;
    unsigned lo, hi;
    chunk_of(blockIdx.x, gridDim.x, n2, &lo, &hi);
    const double hp = vprev ? *hprev : 0.0;
    double a[1] = {0.0};
    double2* w2 = reinterpret_cast<double2*>(w);
    for (unsigned p = lo + threadIdx.x; p < hi; p += blockDim.x) {
        double2 x = w2[p];
        if (vprev) {
            const double2 v = reinterpret_cast<const double2*>(vprev)[p];
            x.x -= hp * v.x;
            x.y -= hp * v.y;
            w2[p] = x;
        }
        if (vnext) {
            const double2 v = reinterpret_cast<const double2*>(vnext)[p];
            a[0] += x.x * v.x + x.y * v.y;
        } else {
            a[0] += x.x * x.x + x.y * x.y;
        }
    }
    if ((n & 1u) && blockIdx.x == gridDim.x - 1 && threadIdx.x == 0) {
        double x = w[n - 1];
        if (vprev) {
            x -= hp * vprev[n - 1];
            w[n - 1] = x;
        }
        a[0] += x * (vnext ? vnext[n - 1] : x);
    }
    block_partials<1>(a, part, gridDim.x, blockIdx.x);
}

void launch_fg_mgs(hipStream_t st, double* w, const double* vprev, const double* hprev, const double* vnext,
                   size_t n, double* part, unsigned* np) {
    const unsigned nb = red_blocks(n / 2 + 1);
    hipLaunchKernelGGL(k_fg_mgs, dim3(nb), dim3(kBlock), 0, st, w, vprev, hprev, vnext, (unsigned)n, part);
    *np = nb;
}

// ---- classical Gram-Schmidt passes of the flexible GMRES --------------------------------
// Dots of w with the NV basis vectors V0 + v * stride (block partials, value v at part[v * nb]),
// and w.w after them with WN. A set gate that reads 0 turns the launch into a no-op.
// A basis vector's 16-byte load; NT marks it streaming (non-temporal): a basis of
// 256^3 grid vectors is read once per pass and is far larger than the caches, and
// keeping it out of them leaves the last-level cache to the vectors that are reused
// (measured: the block solve 35.8 -> 35.2 ms, bitwise the same results).
typedef double FgD2 __attribute__((ext_vector_type(2)));
template <bool NT>
__device__ __forceinline__ double2 fg_basis_load(const double* base, unsigned p) {
    const FgD2* q = reinterpret_cast<const FgD2*>(base) + p;
    FgD2 v;
    if (NT) v = __builtin_nontemporal_load(q);
    else v = *q;
    return double2{v.x, v.y};
}

template <int NV, bool WN, bool NT>
__global__ void __launch_bounds__(kBlock) k_fg_mdot(const double* __restrict__ w, const double* __restrict__ V0,
                                                    size_t stride, unsigned n, double* part, const int* gate) {
    if (gate && !*gate) return;
    constexpr int K = NV + (WN ? 1 : 0);
    const unsigned n2 = n >> 1;
    unsigned lo, hi;
    chunk_of(blockIdx.x, gridDim.x, n2, &lo, &hi);
    double a[K];
#pragma unroll
    for (int k = 0; k < K; ++k) a[k] = 0.0;
    const double2* w2 = reinterpret_cast<const double2*>(w);
    for (unsigned p = lo + threadIdx.x; p < hi; p += blockDim.x) {
        const double2 x = w2[p];
#pragma unroll
        for (int v = 0; v < NV; ++v) {
            const double2 y = fg_basis_load<NT>(V0 + (size_t)v * stride, p);
            a[v] += x.x * y.x + x.y * y.y;
        }
        if (WN) a[K - 1] += x.x * x.x + x.y * x.y;
    }
    if ((n & 1u) && blockIdx.x == gridDim.x - 1 && threadIdx.x == 0) {
        const double x = w[n - 1];
#pragma unroll
        for (int v = 0; v < NV; ++v) a[v] += x * V0[(size_t)v * stride + n - 1];
        if (WN) a[K - 1] += x * x;
    }
    block_partials<K>(a, part, gridDim.x, blockIdx.x);
}

// out[v] (= or +=) the sum of value v's partials, v < nv; *wn = the last value's sum with wn.
__global__ void __launch_bounds__(kFinBlock) k_fg_mfin(const double* __restrict__ part, unsigned np, int nv,
                                                      double* out, double* wn, const int* gate) {
    if (gate && !*gate) return;
    for (int v = 0; v < nv; ++v) {
        const double sv = fin_sum(part + (size_t)v * np, np);
        if (threadIdx.x == 0) out[v] = sv;
    }
    if (wn) {
        const double sw = fin_sum(part + (size_t)nv * np, np);
        if (threadIdx.x == 0) *wn = sw;
    }
}

// w -= sum_v h[v] v_v over the m basis vectors (in order), partials of the new w.w.
template <bool NT>
__global__ void __launch_bounds__(kBlock) k_fg_mupdate(double* __restrict__ w, const double* __restrict__ V0,
                                                       size_t stride, unsigned n, const double* __restrict__ h,
                                                       int m, double* part, const int* gate) {
    if (gate && !*gate) return;
    __shared__ double hs[kFgMaxRestart];
    for (int k = threadIdx.x; k < m; k += blockDim.x) hs[k] = h[k];
    __syncthreads();
    const unsigned n2 = n >> 1;
    unsigned lo, hi;
    chunk_of(blockIdx.x, gridDim.x, n2, &lo, &hi);
    double a[1] = {0.0};
    double2* w2 = reinterpret_cast<double2*>(w);
    for (unsigned p = lo + threadIdx.x; p < hi; p += blockDim.x) {
        double2 x = w2[p];
        for (int v = 0; v < m; ++v) {
            const double2 y = fg_basis_load<NT>(V0 + (size_t)v * stride, p);
            x.x -= hs[v] * y.x;
            x.y -= hs[v] * y.y;
        }
        w2[p] = x;
        a[0] += x.x * x.x + x.y * x.y;
    }
    if ((n & 1u) && blockIdx.x == gridDim.x - 1 && threadIdx.x == 0) {
        double x = w[n - 1];
        for (int v = 0; v < m; ++v) x -= hs[v] * V0[(size_t)v * stride + n - 1];
        w[n - 1] = x;
        a[0] += x * x;
    }
    block_partials<1>(a, part, gridDim.x, blockIdx.x);
}

// *hout = |w| from the update's partials. First pass (add == null): *redo = 1 when |w|^2 fell
// below eta2 * *pre2 (w lost most of its length to the projection, so the rounding left in
// it is relatively large). Second pass (gated by redo): col[v] += add[v], v < m.
__global__ void __launch_bounds__(kFinBlock) k_fg_norm(const double* __restrict__ part, unsigned np, double* hout,
                                                      const double* pre2, double eta2, int* redo, double* col,
                                                      const double* add, int m, const int* gate) {
    if (gate && !*gate) return;
    const double s = fin_sum(part, np);
    if (threadIdx.x == 0) {
        *hout = sqrt(s);
        if (!add) *redo = s < eta2 * *pre2 ? 1 : 0;
    }
    if (add)
        for (int v = threadIdx.x; v < m; v += blockDim.x) col[v] += add[v];
}

namespace {
template <int NV>
void mdot_launch(hipStream_t st, bool wn, unsigned nb, const double* w, const double* V0, size_t stride, unsigned n,
                 double* part, const int* gate) {
    if (wn) hipLaunchKernelGGL((k_fg_mdot<NV, true, true>), dim3(nb), dim3(kBlock), 0, st, w, V0, stride, n, part, gate);
    else hipLaunchKernelGGL((k_fg_mdot<NV, false, true>), dim3(nb), dim3(kBlock), 0, st, w, V0, stride, n, part, gate);
}
}  // namespace

unsigned fg_cgs_blocks(size_t n) { return red_blocks(n / 2 + 1); }

void launch_fg_cgs_dots(hipStream_t st, const double* w, const double* V, size_t stride, size_t n, int m, int group,
                        double* out, double* wn2, double* part, const int* gate) {
    const unsigned nb = fg_cgs_blocks(n);
    for (int g0 = 0; g0 < m; g0 += group) {
        const int nv = m - g0 < group ? m - g0 : group;
        const bool wn = g0 == 0 && wn2;
        const double* V0 = V + (size_t)g0 * stride;
        switch (nv) {
            case 1: mdot_launch<1>(st, wn, nb, w, V0, stride, (unsigned)n, part, gate); break;
            case 2: mdot_launch<2>(st, wn, nb, w, V0, stride, (unsigned)n, part, gate); break;
            case 3: mdot_launch<3>(st, wn, nb, w, V0, stride, (unsigned)n, part, gate); break;
            case 4: mdot_launch<4>(st, wn, nb, w, V0, stride, (unsigned)n, part, gate); break;
            case 5: mdot_launch<5>(st, wn, nb, w, V0, stride, (unsigned)n, part, gate); break;
            case 6: mdot_launch<6>(st, wn, nb, w, V0, stride, (unsigned)n, part, gate); break;
            case 7: mdot_launch<7>(st, wn, nb, w, V0, stride, (unsigned)n, part, gate); break;
            default: mdot_launch<8>(st, wn, nb, w, V0, stride, (unsigned)n, part, gate); break;
        }
        hipLaunchKernelGGL(k_fg_mfin, dim3(1), dim3(kFinBlock), 0, st, part, nb, nv, out + g0, wn ? wn2 : nullptr,
                           gate);
    }
}

void launch_fg_cgs_update(hipStream_t st, double* w, const double* V, size_t stride, size_t n, const double* h, int m,
                          double* part, const int* gate, double* hout, const double* pre2, double eta2, int* redo,
                          double* col, const double* add) {
    const unsigned nb = fg_cgs_blocks(n);
    hipLaunchKernelGGL(k_fg_mupdate<true>, dim3(nb), dim3(kBlock), 0, st, w, V, stride, (unsigned)n, h, m, part, gate);
    hipLaunchKernelGGL(k_fg_norm, dim3(1), dim3(kFinBlock), 0, st, part, nb, hout, pre2, eta2, redo, col, add, m,
                       gate);
}

// out = sum of the partials (its square root with take_sqrt)
__global__ void __launch_bounds__(kFinBlock) k_fg_fin(const double* __restrict__ part, unsigned np, double* out,
                                                      int take_sqrt) {
    const double s = fin_sum(part, np);
    if (threadIdx.x == 0) *out = take_sqrt ? sqrt(s) : s;
}

void launch_fg_fin(hipStream_t st, const double* part, unsigned np, double* out, int take_sqrt) {
    hipLaunchKernelGGL(k_fg_fin, dim3(1), dim3(kFinBlock), 0, st, part, np, out, take_sqrt);
}

// w /= *h (w = 0 when *h is 0: an exact breakdown)
__global__ void __launch_bounds__(kBlock) k_fg_scale(double* __restrict__ w, const double* __restrict__ h,
                                                     unsigned n) {
    const double hv = *h;
    const double inv = hv > 0.0 ? 1.0 / hv : 0.0;
    const unsigned p = blockIdx.x * blockDim.x + threadIdx.x;
    if (2 * p + 1 < n) {
        double2 x = reinterpret_cast<double2*>(w)[p];
        x.x *= inv;
        x.y *= inv;
        reinterpret_cast<double2*>(w)[p] = x;
    } else if (2 * p < n) {
        w[2 * p] *= inv;
    }
}

void launch_fg_scale(hipStream_t st, double* w, const double* h, size_t n) {
    hipLaunchKernelGGL(k_fg_scale, dim3(nblocks((n + 1) / 2)), dim3(kBlock), 0, st, w, h, (unsigned)n);
}

// w *= 1 / *h over the n entries, and block partial sums of the scaled grid part (the
// first ncell entries) into part[block], as k_norm_partials' first component: the sum the
// preconditioner's mean step reads next, without its own pass over w.
__global__ void __launch_bounds__(kBlock) k_fg_scale_sum(double* __restrict__ w, const double* __restrict__ h,
                                                         unsigned n, unsigned ncell, double* part) {
    const double hv = *h;
    const double inv = hv > 0.0 ? 1.0 / hv : 0.0;
    unsigned lo, hi;
    chunk_of(blockIdx.x, gridDim.x, n, &lo, &hi);
    double a[1] = {0.0};
    for (unsigned idx = lo + threadIdx.x; idx < hi; idx += blockDim.x) {
        const double v = w[idx] * inv;
        w[idx] = v;
        if (idx < ncell) a[0] += v;
    }
    block_partials<1>(a, part, gridDim.x, blockIdx.x);
}

void launch_fg_scale_sum(hipStream_t st, double* w, const double* h, size_t n, size_t ncell, double* part,
                         unsigned* np) {
    const unsigned nb = red_blocks(n);
    hipLaunchKernelGGL(k_fg_scale_sum, dim3(nb), dim3(kBlock), 0, st, w, h, (unsigned)n, (unsigned)ncell, part);
    *np = nb;
}

// r = b - r (sub) or r = b, with b = [bg; 0]; partials of r.r
__global__ void __launch_bounds__(kBlock) k_fg_resid(double* __restrict__ r, const double* __restrict__ bg,
                                                     unsigned ncell, unsigned n, int sub, double* part, double phi) {
    unsigned lo, hi;
    chunk_of(blockIdx.x, gridDim.x, n, &lo, &hi);
    double a[1] = {0.0};
    for (unsigned i = lo + threadIdx.x; i < hi; i += blockDim.x) {
        const double b = i < ncell ? bg[i] : phi;
        const double v = sub ? b - r[i] : b;
        r[i] = v;
        a[0] += v * v;
    }
    block_partials<1>(a, part, gridDim.x, blockIdx.x);
}

void launch_fg_resid(hipStream_t st, double* r, const double* bg, size_t ncell, size_t n, int sub, double* part,
                     unsigned* np, double phi) {
    const unsigned nb = red_blocks(n);
    hipLaunchKernelGGL(k_fg_resid, dim3(nb), dim3(kBlock), 0, st, r, bg, (unsigned)ncell, (unsigned)n, sub, part,
                       phi);
    *np = nb;
}

// x[i] += sum_j y_j Z_j[off + i] for i < n (Z_j = Z + j * stride, y on the device)
__global__ void __launch_bounds__(kBlock) k_fg_update(double* __restrict__ x, const double* __restrict__ Z,
                                                      size_t stride, size_t off, unsigned n, int k,
                                                      const double* __restrict__ y) {
    const unsigned i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    double acc = x[i];
    for (int j = 0; j < k; ++j) acc += y[j] * Z[(size_t)j * stride + off + i];
    x[i] = acc;
}

void launch_fg_update(hipStream_t st, double* x, const double* Z, size_t stride, size_t off, size_t n, int k,
                      const double* y) {
    if (n == 0 || k == 0) return;
    hipLaunchKernelGGL(k_fg_update, dim3(nblocks(n)), dim3(kBlock), 0, st, x, Z, stride, off, (unsigned)n, k, y);
}

// Column j of the Hessenberg matrix (column-major, leading dimension ld) is
// complete: apply the previous Givens rotations, form rotation j, advance the
// right-hand side g; out[0] = |g[j+1]| (the residual estimate), out[1] = the
// subdiagonal entry before rotation.
__global__ void k_fg_givens(double* Hd, int ld, double* cs, double* sn, double* g, int j, double* out) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    double* col = Hd + (size_t)j * ld;
    for (int i = 0; i < j; ++i) {
        const double a = col[i], b = col[i + 1];
        col[i] = cs[i] * a + sn[i] * b;
        col[i + 1] = -sn[i] * a + cs[i] * b;
    }
    const double a = col[j], b = col[j + 1];
    const double den = sqrt(a * a + b * b);
    cs[j] = den == 0.0 ? 1.0 : a / den;
    sn[j] = den == 0.0 ? 0.0 : b / den;
    out[1] = b;
    col[j] = den;
    col[j + 1] = 0.0;
    g[j + 1] = -sn[j] * g[j];
    g[j] = cs[j] * g[j];
    out[0] = fabs(g[j + 1]);
}

void launch_fg_givens(hipStream_t st, double* Hd, int ld, double* cs, double* sn, double* g, int j, double* out) {
    hipLaunchKernelGGL(k_fg_givens, dim3(1), dim3(64), 0, st, Hd, ld, cs, sn, g, j, out);
}

// g[0] = *beta, g[1..] = 0
__global__ void k_fg_gstart(double* g, int len, const double* beta) {
    for (int i = threadIdx.x; i < len; i += blockDim.x) g[i] = i == 0 ? *beta : 0.0;
}

void launch_fg_gstart(hipStream_t st, double* g, int len, const double* beta) {
    hipLaunchKernelGGL(k_fg_gstart, dim3(1), dim3(256), 0, st, g, len, beta);
}

// y = R^{-1} g for the leading k x k upper triangle R of the rotated Hessenberg matrix
__global__ void k_fg_backsolve(const double* Hd, int ld, const double* g, double* y, int k) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    for (int i = k - 1; i >= 0; --i) {
        double s = g[i];
        for (int j = i + 1; j < k; ++j) s -= Hd[(size_t)j * ld + i] * y[j];
        const double d = Hd[(size_t)i * ld + i];
        y[i] = d != 0.0 ? s / d : 0.0;
    }
}

void launch_fg_backsolve(hipStream_t st, const double* Hd, int ld, const double* g, double* y, int k) {
    hipLaunchKernelGGL(k_fg_backsolve, dim3(1), dim3(64), 0, st, Hd, ld, g, y, k);
}

}  // namespace brd
