// Geometric multigrid kernels for alpha I - D L on red/black-split levels.
//
// The paper uses a library multigrid whose details it does not give
// (arXiv:1306.3159 Sec. III.E, eq. Helmholtz). This V-cycle is: V(2,2)
// red-black Gauss-Seidel (red = (x+y+z) even; pre-smoothing red then black,
// post-smoothing black then red, so the cycle is symmetric for CG),
// full-weighting restriction R = P^T/8, cell-centred trilinear
// prolongation P, rediscretised coarse operators alpha I - D L_{2h} and a
// dense FP64 (pseudo-)inverse on the coarsest grid.
//
// Split layout: cell (x, y, z) of colour c = (x+y+z)&1 lives at index x/2 of
// row (y, z) of array c. For a cell of colour c at half-index i in row
// (y, z), x = 2i + s with s = ((y+z)&1) ^ c; its x-neighbours are the other
// colour at half-indices i-1+s and i+s, and its y/z-neighbours are the other
// colour at half-index i of the neighbouring rows.
#include "launch.hpp"

namespace brd {

template <typename T>
__device__ __forceinline__ T nb_sum(const T* __restrict__ uo, int i, int y, int z, int hx, int ny, int nz, int s) {
    const size_t row = ((size_t)z * ny + y) * hx;
    const int il = wrapi(i - 1 + s, hx), ir = wrapi(i + s, hx);
    const int ym = wrapi(y - 1, ny), yp = wrapi(y + 1, ny), zm = wrapi(z - 1, nz), zp = wrapi(z + 1, nz);
    const T a = uo[row + il] + uo[row + ir];
    const T b = uo[((size_t)z * ny + ym) * hx + i] + uo[((size_t)z * ny + yp) * hx + i];
    const T c = uo[((size_t)zm * ny + y) * hx + i] + uo[((size_t)zp * ny + y) * hx + i];
    return (a + b) + c;
}

// ---------------------------------------------------------------------------
// Fine-level entry: f = r - mean_r (FP64 natural -> T split) and the first red
// half-sweep from a zero initial guess, u_red = f_red / diag (not stored when u0 is
// null: the cycle's opening black sweep then forms it from f).
template <typename T>
__global__ void __launch_bounds__(kBlock) k_enter(const double* __restrict__ r, T* __restrict__ f0,
                                                  T* __restrict__ f1, T* __restrict__ u0, int hx, int ny, int nz,
                                                  double inv_diag, const Scalars* sc) {
    if (sc && sc->done) return;
    const unsigned nh = (unsigned)hx * ny * nz;
    const unsigned idx = xcd_block(blockIdx.x, gridDim.x) * blockDim.x + threadIdx.x;
    if (idx >= nh) return;
    const int i = idx % hx;
    const unsigned t = idx / hx;
    const int y = t % ny, z = t / ny;
    const double m = sc ? sc->mean_r : 0.0;
    const int s0 = (y + z) & 1;                       // x offset of the red cell in this row
    const size_t rowN = ((size_t)z * ny + y) * (2 * hx);
    const double fr = r[rowN + 2 * i + s0] - m;
    const double fb = r[rowN + 2 * i + (s0 ^ 1)] - m;
    f0[idx] = (T)fr;
    f1[idx] = (T)fb;
    if (u0) u0[idx] = (T)((T)fr * (T)inv_diag);  // null: the cycle opens from f
}

template <typename T>
void launch_enter(hipStream_t st, const double* r, T* f0, T* f1, T* u0, int nx, int ny, int nz, double inv_diag,
                  const Scalars* sc) {
    const unsigned nh = (unsigned)(nx / 2) * ny * nz;
    hipLaunchKernelGGL(k_enter<T>, dim3(nblocks(nh)), dim3(kBlock), 0, st, r, f0, f1, u0, nx / 2, ny, nz, inv_diag,
                       sc);
}

// Fine-level entry from the residual of a guess c held in the split layout: f = g - (alpha c
// - D L c) at every cell (FP64 arithmetic on c's values, T split out) and, when u0 is set, the
// first red half-sweep from zero, u_red = f_red / diag, as k_enter of that FP64 residual writes
// them. A spread term's touched cells are rewritten afterwards (k_resid_spread_enter).
template <typename T>
__global__ void __launch_bounds__(kBlock) k_resid_enter(const double* __restrict__ g, const T* __restrict__ c0,
                                                        const T* __restrict__ c1, T* __restrict__ f0,
                                                        T* __restrict__ f1, T* __restrict__ u0, int hx, int ny, int nz,
                                                        double alpha, double s, double inv_diag) {
    const unsigned nh = (unsigned)hx * ny * nz;
    const unsigned idx = xcd_block(blockIdx.x, gridDim.x) * blockDim.x + threadIdx.x;
    if (idx >= nh) return;
    const int i = idx % hx;
    const unsigned t = idx / hx;
    const int y = t % ny, z = t / ny;
    const int s0 = (y + z) & 1;  // x offset of the red cell in this row
    const double fr = split_resid(g, c0, c1, 2 * i + s0, y, z, 2 * hx, ny, nz, alpha, s);
    const double fb = split_resid(g, c0, c1, 2 * i + (s0 ^ 1), y, z, 2 * hx, ny, nz, alpha, s);
    f0[idx] = (T)fr;
    f1[idx] = (T)fb;
    if (u0) u0[idx] = (T)((T)fr * (T)inv_diag);
}

template <typename T>
void launch_resid_enter(hipStream_t st, const double* g, const T* c0, const T* c1, T* f0, T* f1, T* u0, int nx,
                        int ny, int nz, double alpha, double s, double inv_diag) {
    const unsigned nh = (unsigned)(nx / 2) * ny * nz;
    hipLaunchKernelGGL(k_resid_enter<T>, dim3(nblocks(nh)), dim3(kBlock), 0, st, g, c0, c1, f0, f1, u0, nx / 2, ny,
                       nz, alpha, s, inv_diag);
}

// ---------------------------------------------------------------------------
// Gauss-Seidel half-sweep on colour `color`: u_c = (f_c + s * sum nbrs) / diag.
template <typename T>
__global__ void __launch_bounds__(kMaxTuneBlock) k_gs(T* __restrict__ uc, const T* __restrict__ uo,
                                               const T* __restrict__ fc, int hx, int ny, int nz, int color, T s,
                                               T inv_diag, const Scalars* sc) {
    if (sc && sc->done) return;
    const unsigned nh = (unsigned)hx * ny * nz;
    const unsigned idx = xcd_block(blockIdx.x, gridDim.x) * blockDim.x + threadIdx.x;
    if (idx >= nh) return;
    const int i = idx % hx;
    const unsigned t = idx / hx;
    const int y = t % ny, z = t / ny;
    const int so = ((y + z) & 1) ^ color;
    const T nb = nb_sum(uo, i, y, z, hx, ny, nz, so);
    uc[idx] = (fc[idx] + s * nb) * inv_diag;
}

// Vector form: each thread updates VW = 16 / sizeof(T) consecutive cells of a
// split row with 16-byte loads and stores (same arithmetic and summation
// order as k_gs, so results are bitwise identical). Needs hx % VW == 0.
template <typename T>
struct VecOf;
template <>
struct VecOf<float> {
    typedef float type __attribute__((ext_vector_type(4)));
    static constexpr int W = 4;
};
template <>
struct VecOf<double> {
    typedef double type __attribute__((ext_vector_type(2)));
    static constexpr int W = 2;
};

// x-neighbours of the VW cells starting at i0 (x offset so): left = other[i-1+so], right = other[i+so]
template <typename T>
__device__ __forceinline__ void row_neighbours(const T* __restrict__ orow, int i0, int hx, int so,
                                               typename VecOf<T>::type& left, typename VecOf<T>::type& right) {
    typedef typename VecOf<T>::type V;
    constexpr int VW = VecOf<T>::W;
    const V o = *reinterpret_cast<const V*>(orow + i0);
    const T edge = so ? orow[i0 + VW == hx ? 0 : i0 + VW] : orow[i0 == 0 ? hx - 1 : i0 - 1];
#pragma unroll
    for (int k = 0; k < VW; ++k) {
        left[k] = so ? o[k] : (k ? o[k - 1] : edge);
        right[k] = so ? (k + 1 < VW ? o[k + 1] : edge) : o[k];
    }
}

// FROM_F: the first half-sweep after a V-cycle entry whose other colour still holds its
// zero-guess sweep u = f / diag; uo is then that colour's f, scaled on the fly (the same
// product the entry would have stored), so the entry need not store it.
template <typename T, bool FROM_F = false>
__device__ __forceinline__ void gs_vec_body(T* __restrict__ uc, const T* __restrict__ uo, const T* __restrict__ fc, int hx, int ny, int nz, int color, T s, T inv_diag, Blk blk) {
    typedef typename VecOf<T>::type V;
    constexpr int VW = VecOf<T>::W;
    const int hv = hx / VW;
    const unsigned nv = (unsigned)hv * ny * nz;
    const unsigned idx = xcd_block(blk.b, blk.nb) * blockDim.x + threadIdx.x;
    if (idx >= nv) return;
    const int iv = idx % hv;
    const unsigned t = idx / hv;
    const int y = t % ny, z = t / ny;
    const int i0 = iv * VW;
    const int so = ((y + z) & 1) ^ color;
    const size_t row = ((size_t)z * ny + y) * hx;
    V left, right;
    row_neighbours<T>(uo + row, i0, hx, so, left, right);
    const V ym = *reinterpret_cast<const V*>(uo + ((size_t)z * ny + wrapi(y - 1, ny)) * hx + i0);
    const V yp = *reinterpret_cast<const V*>(uo + ((size_t)z * ny + wrapi(y + 1, ny)) * hx + i0);
    const V zm = *reinterpret_cast<const V*>(uo + ((size_t)wrapi(z - 1, nz) * ny + y) * hx + i0);
    const V zp = *reinterpret_cast<const V*>(uo + ((size_t)wrapi(z + 1, nz) * ny + y) * hx + i0);
    const V f = *reinterpret_cast<const V*>(fc + row + i0);
    V out;
    if (FROM_F) {
#pragma unroll
        for (int k = 0; k < VW; ++k) {
            // each scaled value rounded on its own, as the entry's stored sweep is
            T l, r, a, b, c, e;
            {
#pragma clang fp contract(off)
                l = left[k] * inv_diag;
                r = right[k] * inv_diag;
                a = ym[k] * inv_diag;
                b = yp[k] * inv_diag;
                c = zm[k] * inv_diag;
                e = zp[k] * inv_diag;
            }
            out[k] = (f[k] + s * (((l + r) + (a + b)) + (c + e))) * inv_diag;
        }
    } else {
#pragma unroll
        for (int k = 0; k < VW; ++k)
            out[k] = (f[k] + s * (((left[k] + right[k]) + (ym[k] + yp[k])) + (zm[k] + zp[k]))) * inv_diag;
    }
    *reinterpret_cast<V*>(uc + row + i0) = out;
}

template <typename T>
__global__ void __launch_bounds__(kMaxTuneBlock) k_gs_vec(T* __restrict__ uc, const T* __restrict__ uo,
                                                   const T* __restrict__ fc, int hx, int ny, int nz, int color, T s,
                                                   T inv_diag, const Scalars* sc) {
    if (sc && sc->done) return;
    gs_vec_body<T>(uc, uo, fc, hx, ny, nz, color, s, inv_diag, Blk{blockIdx.x, gridDim.x});
}

template <typename T>
__global__ void __launch_bounds__(kMaxTuneBlock) k_gs_vec_from_f(T* __restrict__ uc, const T* __restrict__ fo,
                                                          const T* __restrict__ fc, int hx, int ny, int nz,
                                                          int color, T s, T inv_diag, const Scalars* sc) {
    if (sc && sc->done) return;
    gs_vec_body<T, true>(uc, fo, fc, hx, ny, nz, color, s, inv_diag, Blk{blockIdx.x, gridDim.x});
}

// The closing red half-sweep on the finest level fused with the CG dots of
// its result z: block partials (sum z, z.r, z.q) over both colours, r and q
// natural FP64 (split index i of a row is the natural cell pair 2i, 2i + 1).
// The black z at the thread's split indices are the x-neighbour vector the
// sweep loads anyway. Needs hx % VW == 0 and a non-null sc.
template <typename T>
__device__ __forceinline__ void gs_vec_dots_body(T* __restrict__ uc, const T* __restrict__ uo, const T* __restrict__ fc, int hx, int ny, int nz, T s, T inv_diag, const double* __restrict__ r, const double* __restrict__ q, double* part, Blk blk) {
    typedef typename VecOf<T>::type V;
    typedef typename VecOf<double>::type D2;
    constexpr int VW = VecOf<T>::W;
    const int hv = hx / VW;
    const unsigned nv = (unsigned)hv * ny * nz;
    const unsigned idx = xcd_block(blk.b, blk.nb) * blockDim.x + threadIdx.x;
    double acc[3] = {0.0, 0.0, 0.0};
    if (idx < nv) {
        const int iv = idx % hv;
        const unsigned t = idx / hv;
        const int y = t % ny, z = t / ny;
        const int i0 = iv * VW;
        const int par = (y + z) & 1;  // red cells sit at x = 2i + par; the even cell's colour is par
        const size_t row = ((size_t)z * ny + y) * hx;
        V left, right;
        row_neighbours<T>(uo + row, i0, hx, par, left, right);
        const V blk = *reinterpret_cast<const V*>(uo + row + i0);
        const V ym = *reinterpret_cast<const V*>(uo + ((size_t)z * ny + wrapi(y - 1, ny)) * hx + i0);
        const V yp = *reinterpret_cast<const V*>(uo + ((size_t)z * ny + wrapi(y + 1, ny)) * hx + i0);
        const V zm = *reinterpret_cast<const V*>(uo + ((size_t)wrapi(z - 1, nz) * ny + y) * hx + i0);
        const V zp = *reinterpret_cast<const V*>(uo + ((size_t)wrapi(z + 1, nz) * ny + y) * hx + i0);
        const V f = *reinterpret_cast<const V*>(fc + row + i0);
        V out;
#pragma unroll
        for (int k = 0; k < VW; ++k)
            out[k] = (f[k] + s * (((left[k] + right[k]) + (ym[k] + yp[k])) + (zm[k] + zp[k]))) * inv_diag;
        *reinterpret_cast<V*>(uc + row + i0) = out;
#pragma unroll
        for (int k = 0; k < VW; ++k) {
            const double zr = (double)out[k], zb = (double)blk[k];
            const double za = par ? zb : zr, zc = par ? zr : zb;  // even, odd cell
            const D2 rv = reinterpret_cast<const D2*>(r)[row + i0 + k];
            const D2 qv = reinterpret_cast<const D2*>(q)[row + i0 + k];
            acc[0] += za + zc;
            acc[1] += za * rv[0] + zc * rv[1];
            acc[2] += za * qv[0] + zc * qv[1];
        }
    }
    block_partials<3>(acc, part, blk.nb, blk.b);
}

template <typename T>
__global__ void __launch_bounds__(kMaxTuneBlock) k_gs_vec_dots(T* __restrict__ uc, const T* __restrict__ uo,
                                                        const T* __restrict__ fc, int hx, int ny, int nz, T s,
                                                        T inv_diag, const double* __restrict__ r,
                                                        const double* __restrict__ q, double* part,
                                                        const Scalars* sc) {
    if (sc->done) return;
    gs_vec_dots_body<T>(uc, uo, fc, hx, ny, nz, s, inv_diag, r, q, part, Blk{blockIdx.x, gridDim.x});
}

// Returns the number of partial slots, or 0 when the level is not vectorizable
// (nothing launched: the caller sweeps with launch_gs and forms the dots apart).
template <typename T>
unsigned launch_gs_dots(hipStream_t st, T* uc, const T* uo, const T* fc, int hx, int ny, int nz, double s,
                        double inv_diag, const double* r, const double* q, double* part, const Scalars* sc, int bs) {
    constexpr int VW = VecOf<T>::W;
    if (hx % VW != 0 || hx < VW) return 0;
    const unsigned nv = (unsigned)(hx / VW) * ny * nz;
    const unsigned nb = nblocks(nv, bs);
    hipLaunchKernelGGL(k_gs_vec_dots<T>, dim3(nb), dim3(bs), 0, st, uc, uo, fc, hx, ny, nz, (T)s, (T)inv_diag, r, q,
                       part, sc);
    return nb;
}

template <typename T>
bool launch_gs_from_f(hipStream_t st, T* uc, const T* fo, const T* fc, int hx, int ny, int nz, int color, double s,
                      double inv_diag, const Scalars* sc, int bs) {
    constexpr int VW = VecOf<T>::W;
    if (hx % VW != 0 || hx < VW) return false;
    const unsigned nv = (unsigned)(hx / VW) * ny * nz;
    hipLaunchKernelGGL(k_gs_vec_from_f<T>, dim3(nblocks(nv, bs)), dim3(bs), 0, st, uc, fo, fc, hx, ny, nz, color,
                       (T)s, (T)inv_diag, sc);
    return true;
}

template <typename T>
void launch_gs(hipStream_t st, T* uc, const T* uo, const T* fc, int hx, int ny, int nz, int color, double s,
               double inv_diag, const Scalars* sc, int bs) {
    constexpr int VW = VecOf<T>::W;
    if (hx % VW == 0 && hx >= VW) {
        const unsigned nv = (unsigned)(hx / VW) * ny * nz;
        hipLaunchKernelGGL(k_gs_vec<T>, dim3(nblocks(nv, bs)), dim3(bs), 0, st, uc, uo, fc, hx, ny, nz, color, (T)s,
                           (T)inv_diag, sc);
        return;
    }
    const unsigned nh = (unsigned)hx * ny * nz;
    hipLaunchKernelGGL(k_gs<T>, dim3(nblocks(nh, bs)), dim3(bs), 0, st, uc, uo, fc, hx, ny, nz, color, (T)s,
                       (T)inv_diag, sc);
}

// ---------------------------------------------------------------------------
// Residual after pre-smoothing. The pre-smoothing sweeps end with a black
// half-sweep, after which the black residual f - (diag u - s sum nbrs) is zero
// in exact arithmetic: only the red residual is formed (split array r0), and
// the restriction takes the black cells as zero.
template <typename T>
__global__ void __launch_bounds__(kMaxTuneBlock) k_resid(const T* __restrict__ u0, const T* __restrict__ u1,
                                                  const T* __restrict__ f0, T* __restrict__ r0, int hx, int ny,
                                                  int nz, T s, T diag, const Scalars* sc) {
    if (sc && sc->done) return;
    const unsigned nh = (unsigned)hx * ny * nz;
    const unsigned idx = xcd_block(blockIdx.x, gridDim.x) * blockDim.x + threadIdx.x;
    if (idx >= nh) return;
    const int i = idx % hx;
    const unsigned t = idx / hx;
    const int y = t % ny, z = t / ny;
    const T nr = nb_sum(u1, i, y, z, hx, ny, nz, (y + z) & 1);  // neighbours of a red cell are black
    r0[idx] = f0[idx] - (diag * u0[idx] - s * nr);
}

template <typename T>
__device__ __forceinline__ void resid_vec_body(const T* __restrict__ u0, const T* __restrict__ u1, const T* __restrict__ f0, T* __restrict__ r0, int hx, int ny, int nz, T s, T diag, Blk blk) {
    typedef typename VecOf<T>::type V;
    constexpr int VW = VecOf<T>::W;
    const int hv = hx / VW;
    const unsigned nv = (unsigned)hv * ny * nz;
    const unsigned idx = xcd_block(blk.b, blk.nb) * blockDim.x + threadIdx.x;
    if (idx >= nv) return;
    const int iv = idx % hv;
    const unsigned t = idx / hv;
    const int y = t % ny, z = t / ny;
    const int i0 = iv * VW;
    const size_t row = ((size_t)z * ny + y) * hx;
    V left, right;
    row_neighbours<T>(u1 + row, i0, hx, (y + z) & 1, left, right);
    const V ym = *reinterpret_cast<const V*>(u1 + ((size_t)z * ny + wrapi(y - 1, ny)) * hx + i0);
    const V yp = *reinterpret_cast<const V*>(u1 + ((size_t)z * ny + wrapi(y + 1, ny)) * hx + i0);
    const V zm = *reinterpret_cast<const V*>(u1 + ((size_t)wrapi(z - 1, nz) * ny + y) * hx + i0);
    const V zp = *reinterpret_cast<const V*>(u1 + ((size_t)wrapi(z + 1, nz) * ny + y) * hx + i0);
    const V u = *reinterpret_cast<const V*>(u0 + row + i0);
    const V f = *reinterpret_cast<const V*>(f0 + row + i0);
    V out;
#pragma unroll
    for (int k = 0; k < VW; ++k)
        out[k] = f[k] - (diag * u[k] - s * (((left[k] + right[k]) + (ym[k] + yp[k])) + (zm[k] + zp[k])));
    *reinterpret_cast<V*>(r0 + row + i0) = out;
}

template <typename T>
__global__ void __launch_bounds__(kMaxTuneBlock) k_resid_vec(const T* __restrict__ u0, const T* __restrict__ u1,
                                                      const T* __restrict__ f0, T* __restrict__ r0, int hx, int ny,
                                                      int nz, T s, T diag, const Scalars* sc) {
    if (sc && sc->done) return;
    resid_vec_body<T>(u0, u1, f0, r0, hx, ny, nz, s, diag, Blk{blockIdx.x, gridDim.x});
}

template <typename T>
void launch_resid_red(hipStream_t st, const T* u0, const T* u1, const T* f0, T* r0, int hx, int ny, int nz, double s,
                      double diag, const Scalars* sc, int bs) {
    constexpr int VW = VecOf<T>::W;
    if (hx % VW == 0 && hx >= VW) {
        const unsigned nv = (unsigned)(hx / VW) * ny * nz;
        hipLaunchKernelGGL(k_resid_vec<T>, dim3(nblocks(nv, bs)), dim3(bs), 0, st, u0, u1, f0, r0, hx, ny, nz, (T)s,
                           (T)diag, sc);
        return;
    }
    const unsigned nh = (unsigned)hx * ny * nz;
    hipLaunchKernelGGL(k_resid<T>, dim3(nblocks(nh, bs)), dim3(bs), 0, st, u0, u1, f0, r0, hx, ny, nz, (T)s, (T)diag,
                       sc);
}

// ---------------------------------------------------------------------------
// Full-weighting restriction, 1-D weights (1, 3, 3, 1)/8 over fine cells
// 2X-1 .. 2X+2, of the red residual r0 (black cells zero). Writes the coarse
// right-hand side in split layout together with the zero-guess red
// half-sweep, or in natural layout on the coarsest level.
//
// In a fine row of parity p = (y + z) & 1 the red cells are x = 2i + p, so
// of the four fine cells of coarse X the red ones are 2X-1 (weight 1/8) and
// 2X+1 (3/8) when p = 1, 2X (3/8) and 2X+2 (1/8) when p = 0.
template <typename T>
__device__ __forceinline__ T restrict_row(T w0, T w1, int p, T a, T b, T c) {
    // p = 1: (a, b) = r0[X-1], r0[X]; p = 0: (b, c) = r0[X], r0[X+1]
    return p ? w0 * a + w1 * b : w1 * b + w0 * c;
}

template <typename T>
__global__ void __launch_bounds__(kMaxTuneBlock) k_restrict(const T* __restrict__ r0, int nx, int ny, int nz,
                                                     T* __restrict__ cf0, T* __restrict__ cf1, T* __restrict__ cu0,
                                                     int coarse_natural, T inv_diag_c, const Scalars* sc) {
    if (sc && sc->done) return;
    const int cx = nx >> 1, cy = ny >> 1, cz = nz >> 1;
    const unsigned nc = (unsigned)cx * cy * cz;
    const unsigned idx = xcd_block(blockIdx.x, gridDim.x) * blockDim.x + threadIdx.x;
    if (idx >= nc) return;
    const int X = idx % cx;
    const unsigned t = idx / cx;
    const int Y = t % cy, Z = t / cy;
    const int hx = nx >> 1;
    const T w0 = (T)0.125, w1 = (T)0.375;
    const int xl = X == 0 ? hx - 1 : X - 1, xr = X + 1 == hx ? 0 : X + 1;
    T acc = 0;
#pragma unroll
    for (int c = 0; c < 4; ++c) {
        const int z = wrapi(2 * Z - 1 + c, nz);
        T accb = 0;
#pragma unroll
        for (int b = 0; b < 4; ++b) {
            const int y = wrapi(2 * Y - 1 + b, ny);
            const T* row = r0 + ((size_t)z * ny + y) * hx;
            const int p = (y + z) & 1;
            accb += (b == 0 || b == 3 ? w0 : w1) * restrict_row(w0, w1, p, p ? row[xl] : (T)0, row[X], p ? (T)0 : row[xr]);
        }
        acc += (c == 0 || c == 3 ? w0 : w1) * accb;
    }
    if (coarse_natural) {
        cf0[idx] = acc;
    } else {
        const size_t j = ((size_t)Z * cy + Y) * (cx >> 1) + (X >> 1);
        if ((X + Y + Z) & 1) {
            cf1[j] = acc;
        } else {
            cf0[j] = acc;
            cu0[j] = acc * inv_diag_c;
        }
    }
}

// Four consecutive coarse cells per thread: one 4-wide load of r0 per fine
// row plus its two edge values; same arithmetic as k_restrict. Needs cx % 4 == 0.
template <typename T>
__device__ __forceinline__ void restrict4_body(const T* __restrict__ r0, int nx, int ny, int nz, T* __restrict__ cf0, T* __restrict__ cf1, T* __restrict__ cu0, int coarse_natural, T inv_diag_c, Blk blk) {
    typedef T V4 __attribute__((ext_vector_type(4)));
    typedef T V2 __attribute__((ext_vector_type(2)));
    const int cx = nx >> 1, cy = ny >> 1, cz = nz >> 1, cv = cx >> 2;
    const unsigned n4 = (unsigned)cv * cy * cz;
    const unsigned idx = xcd_block(blk.b, blk.nb) * blockDim.x + threadIdx.x;
    if (idx >= n4) return;
    const int v = idx % cv;
    const unsigned t = idx / cv;
    const int Y = t % cy, Z = t / cy;
    const int hx = nx >> 1, X0 = 4 * v;
    const T w0 = (T)0.125, w1 = (T)0.375;
    const int xl = X0 == 0 ? hx - 1 : X0 - 1, xr = X0 + 4 == hx ? 0 : X0 + 4;
    T acc[4] = {0, 0, 0, 0};
#pragma unroll
    for (int c = 0; c < 4; ++c) {
        const int z = wrapi(2 * Z - 1 + c, nz);
        T accb[4] = {0, 0, 0, 0};
#pragma unroll
        for (int b = 0; b < 4; ++b) {
            const int y = wrapi(2 * Y - 1 + b, ny);
            const T* row = r0 + ((size_t)z * ny + y) * hx;
            const int p = (y + z) & 1;
            const V4 m = *reinterpret_cast<const V4*>(row + X0);
            const T e = p ? row[xl] : row[xr];
            const T wb = (b == 0 || b == 3) ? w0 : w1;
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                const T a = p ? (k ? m[k - 1] : e) : (T)0;
                const T cc = p ? (T)0 : (k < 3 ? m[k + 1] : e);
                accb[k] += wb * restrict_row(w0, w1, p, a, m[k], cc);
            }
        }
        const T wc = (c == 0 || c == 3) ? w0 : w1;
#pragma unroll
        for (int k = 0; k < 4; ++k) acc[k] += wc * accb[k];
    }
    if (coarse_natural) {
        *reinterpret_cast<V4*>(cf0 + ((size_t)Z * cy + Y) * cx + X0) = V4{acc[0], acc[1], acc[2], acc[3]};
    } else {
        const int pc = (Y + Z) & 1;  // coarse X0 is red when pc == 0
        const size_t j = ((size_t)Z * cy + Y) * (cx >> 1) + (X0 >> 1);
        const V2 red = pc ? V2{acc[1], acc[3]} : V2{acc[0], acc[2]};
        const V2 blk = pc ? V2{acc[0], acc[2]} : V2{acc[1], acc[3]};
        *reinterpret_cast<V2*>(cf0 + j) = red;
        *reinterpret_cast<V2*>(cf1 + j) = blk;
        *reinterpret_cast<V2*>(cu0 + j) = red * inv_diag_c;
    }
}

// The same restriction for a 4 x 2 x 2 block of coarse cells per thread (X0 .. X0+3,
// Y0 .. Y0+1, Z0 .. Z0+1): the block's six fine z-planes by six fine y-rows are read once
// (36 row reads for 16 cells instead of 64), and every cell sums its terms in the order of
// restrict4_body (its four y-rows of a plane, then its four planes), so the results are
// bitwise those of the one-row form.
template <typename T>
__device__ __forceinline__ void restrict4q_body(const T* __restrict__ r0, int nx, int ny, int nz, T* __restrict__ cf0,
                                                T* __restrict__ cf1, T* __restrict__ cu0, int coarse_natural,
                                                T inv_diag_c, Blk blk) {
    typedef T V4 __attribute__((ext_vector_type(4)));
    typedef T V2 __attribute__((ext_vector_type(2)));
    const int cx = nx >> 1, cy = ny >> 1, cz = nz >> 1, cv = cx >> 2, qy = cy >> 1;
    const unsigned nq = (unsigned)cv * qy * (cz >> 1);
    const unsigned idx = xcd_block(blk.b, blk.nb) * blockDim.x + threadIdx.x;
    if (idx >= nq) return;
    const int v = idx % cv;
    const unsigned t = idx / cv;
    const int Y0 = 2 * (int)(t % qy), Z0 = 2 * (int)(t / qy);
    const int hx = nx >> 1, X0 = 4 * v;
    const T w0 = (T)0.125, w1 = (T)0.375;
    const int xl = X0 == 0 ? hx - 1 : X0 - 1, xr = X0 + 4 == hx ? 0 : X0 + 4;
    T acc[2][2][4] = {};
#pragma unroll
    for (int cc = 0; cc < 6; ++cc) {  // fine z = 2 Z0 - 1 + cc: plane cc of cell Z0, cc - 2 of Z0 + 1
        const int z = wrapi(2 * Z0 - 1 + cc, nz);
        T accb[2][4] = {};
#pragma unroll
        for (int bb = 0; bb < 6; ++bb) {  // fine y = 2 Y0 - 1 + bb: row bb of cell Y0, bb - 2 of Y0 + 1
            const int y = wrapi(2 * Y0 - 1 + bb, ny);
            const T* row = r0 + ((size_t)z * ny + y) * hx;
            const int p = (y + z) & 1;
            const V4 m = *reinterpret_cast<const V4*>(row + X0);
            const T e = p ? row[xl] : row[xr];
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                const T a = p ? (k ? m[k - 1] : e) : (T)0;
                const T c3 = p ? (T)0 : (k < 3 ? m[k + 1] : e);
                const T rr = restrict_row(w0, w1, p, a, m[k], c3);
#pragma unroll
                for (int yo = 0; yo < 2; ++yo) {
                    const int b = bb - 2 * yo;
                    if (b >= 0 && b < 4) accb[yo][k] += ((b == 0 || b == 3) ? w0 : w1) * rr;
                }
            }
        }
#pragma unroll
        for (int zo = 0; zo < 2; ++zo) {
            const int c = cc - 2 * zo;
            if (c < 0 || c >= 4) continue;
            const T wc = (c == 0 || c == 3) ? w0 : w1;
#pragma unroll
            for (int yo = 0; yo < 2; ++yo)
#pragma unroll
                for (int k = 0; k < 4; ++k) acc[zo][yo][k] += wc * accb[yo][k];
        }
    }
#pragma unroll
    for (int zo = 0; zo < 2; ++zo)
#pragma unroll
        for (int yo = 0; yo < 2; ++yo) {
            const int Y = Y0 + yo, Z = Z0 + zo;
            const T* a4 = acc[zo][yo];
            if (coarse_natural) {
                *reinterpret_cast<V4*>(cf0 + ((size_t)Z * cy + Y) * cx + X0) = V4{a4[0], a4[1], a4[2], a4[3]};
            } else {
                const int pc = (Y + Z) & 1;  // coarse X0 is red when pc == 0
                const size_t j = ((size_t)Z * cy + Y) * (cx >> 1) + (X0 >> 1);
                const V2 red = pc ? V2{a4[1], a4[3]} : V2{a4[0], a4[2]};
                const V2 blk = pc ? V2{a4[0], a4[2]} : V2{a4[1], a4[3]};
                *reinterpret_cast<V2*>(cf0 + j) = red;
                *reinterpret_cast<V2*>(cf1 + j) = blk;
                *reinterpret_cast<V2*>(cu0 + j) = red * inv_diag_c;
            }
        }
}

template <typename T>
__global__ void __launch_bounds__(kMaxTuneBlock) k_restrict4q(const T* __restrict__ r0, int nx, int ny, int nz,
                                                       T* __restrict__ cf0, T* __restrict__ cf1, T* __restrict__ cu0,
                                                       int coarse_natural, T inv_diag_c, const Scalars* sc) {
    if (sc && sc->done) return;
    restrict4q_body<T>(r0, nx, ny, nz, cf0, cf1, cu0, coarse_natural, inv_diag_c, Blk{blockIdx.x, gridDim.x});
}

template <typename T>
__global__ void __launch_bounds__(kMaxTuneBlock) k_restrict4(const T* __restrict__ r0, int nx, int ny, int nz,
                                                      T* __restrict__ cf0, T* __restrict__ cf1, T* __restrict__ cu0,
                                                      int coarse_natural, T inv_diag_c, const Scalars* sc) {
    if (sc && sc->done) return;
    restrict4_body<T>(r0, nx, ny, nz, cf0, cf1, cu0, coarse_natural, inv_diag_c, Blk{blockIdx.x, gridDim.x});
}

template <typename T>
void launch_restrict(hipStream_t st, const T* r0, int nx, int ny, int nz, T* cf0, T* cf1, T* cu0, int coarse_natural,
                     double inv_diag_c, const Scalars* sc, int bs) {
    const int cx = nx / 2;
    if constexpr (sizeof(T) == 4) {  // the FP64 block would not fit in registers
        if (cx % 4 == 0 && (ny / 2) % 2 == 0 && (nz / 2) % 2 == 0) {
            const unsigned nq = (unsigned)(cx / 4) * (ny / 4) * (nz / 4);
            hipLaunchKernelGGL(k_restrict4q<T>, dim3(nblocks(nq, bs)), dim3(bs), 0, st, r0, nx, ny, nz, cf0, cf1,
                               cu0, coarse_natural, (T)inv_diag_c, sc);
            return;
        }
    }
    if (cx % 4 == 0) {
        const unsigned n4 = (unsigned)(cx / 4) * (ny / 2) * (nz / 2);
        hipLaunchKernelGGL(k_restrict4<T>, dim3(nblocks(n4, bs)), dim3(bs), 0, st, r0, nx, ny, nz, cf0, cf1, cu0,
                           coarse_natural, (T)inv_diag_c, sc);
        return;
    }
    const unsigned nc = (unsigned)cx * (ny / 2) * (nz / 2);
    hipLaunchKernelGGL(k_restrict<T>, dim3(nblocks(nc, bs)), dim3(bs), 0, st, r0, nx, ny, nz, cf0, cf1, cu0,
                       coarse_natural, (T)inv_diag_c, sc);
}

// ---------------------------------------------------------------------------
// Trilinear prolongation added to the fine split level: fine x = 2I + s takes
// 3/4 of coarse I and 1/4 of coarse I-1 (s = 0) or I+1 (s = 1) per axis.
template <typename T>
__device__ __forceinline__ T coarse_at(const T* __restrict__ c0, const T* __restrict__ c1, int nat, int X, int Y,
                                       int Z, int cx, int cy) {
    if (nat) return c0[((size_t)Z * cy + Y) * cx + X];
    const size_t j = ((size_t)Z * cy + Y) * (cx >> 1) + (X >> 1);
    return ((X + Y + Z) & 1) ? c1[j] : c0[j];
}

// u plus the trilinear correction of one fine cell from its four coarse rows (J0, K0),
// (J1, K0), (J0, K1), (J1, K1): m is a row's value at the cell's own coarse x, n the one at
// the neighbour on the cell's side. Evaluated as written, with no contraction beyond the
// explicit FMAs, so that every form of the correction (per level, blocked, LDS tail) rounds
// alike.
template <typename T>
__device__ __forceinline__ T tri_add(T u, T m00, T n00, T m10, T n10, T m01, T n01, T m11, T n11) {
#pragma clang fp contract(off)
    const T a00 = fma((T)0.75, m00, (T)0.25 * n00);
    const T a10 = fma((T)0.75, m10, (T)0.25 * n10);
    const T a01 = fma((T)0.75, m01, (T)0.25 * n01);
    const T a11 = fma((T)0.75, m11, (T)0.25 * n11);
    const T b0 = fma((T)0.75, a00, (T)0.25 * a10);
    const T b1 = fma((T)0.75, a01, (T)0.25 * a11);
    return u + fma((T)0.75, b0, (T)0.25 * b1);
}

template <typename T>
__global__ void __launch_bounds__(kMaxTuneBlock) k_prolong(const T* __restrict__ cu0, const T* __restrict__ cu1, int nat,
                                                    T* __restrict__ u0, T* __restrict__ u1, int nx, int ny, int nz,
                                                    const Scalars* sc) {
    if (sc && sc->done) return;
    const int hx = nx >> 1;
    const unsigned nh = (unsigned)hx * ny * nz;
    const unsigned idx = xcd_block(blockIdx.x, gridDim.x) * blockDim.x + threadIdx.x;
    if (idx >= nh) return;
    const int i = idx % hx;
    const unsigned t = idx / hx;
    const int y = t % ny, z = t / ny;
    const int cx = nx >> 1, cy = ny >> 1, cz = nz >> 1;
    const int J0 = y >> 1, J1 = wrapi((y & 1) ? J0 + 1 : J0 - 1, cy);
    const int K0 = z >> 1, K1 = wrapi((z & 1) ? K0 + 1 : K0 - 1, cz);
    const int s0 = (y + z) & 1;
#pragma unroll
    for (int c = 0; c < 2; ++c) {
        const int x = 2 * i + (s0 ^ c);
        const int I0 = x >> 1, I1 = wrapi((x & 1) ? I0 + 1 : I0 - 1, cx);
        T* u = c == 0 ? u0 : u1;
        u[idx] = tri_add(u[idx], coarse_at(cu0, cu1, nat, I0, J0, K0, cx, cy),
                         coarse_at(cu0, cu1, nat, I1, J0, K0, cx, cy), coarse_at(cu0, cu1, nat, I0, J1, K0, cx, cy),
                         coarse_at(cu0, cu1, nat, I1, J1, K0, cx, cy), coarse_at(cu0, cu1, nat, I0, J0, K1, cx, cy),
                         coarse_at(cu0, cu1, nat, I1, J0, K1, cx, cy), coarse_at(cu0, cu1, nat, I0, J1, K1, cx, cy),
                         coarse_at(cu0, cu1, nat, I1, J1, K1, cx, cy));
    }
}

// The coarse values c(i0 + d), d = 0 .. VW-1, of row (Y, Z) of a split coarse level, and
// the next one on the fine cells' side, e = c(i0 + VW) (s = 1) or c(i0 - 1) (s = 0), wrapped.
// i0 is a multiple of VW, hence even: c(i0 + d) is element i0/2 + d/2 of c1 when d + Y + Z
// is odd and of c0 otherwise, so one VW/2-wide load from each half gives the run.
template <typename T>
__device__ __forceinline__ void coarse_row(const T* __restrict__ c0, const T* __restrict__ c1, int Y, int Z, int i0,
                                           int s, int cx, int cy, T (&m)[VecOf<T>::W], T& e) {
    constexpr int VW = VecOf<T>::W, HW = VW / 2;
    struct alignas(sizeof(T) * HW) Half { T v[HW]; };
    const size_t rb = ((size_t)Z * cy + Y) * (cx >> 1);
    const int p = (Y + Z) & 1;
    const Half a = *reinterpret_cast<const Half*>(c0 + rb + (i0 >> 1));
    const Half b = *reinterpret_cast<const Half*>(c1 + rb + (i0 >> 1));
#pragma unroll
    for (int d = 0; d < VW; ++d) m[d] = ((d + p) & 1) ? b.v[d >> 1] : a.v[d >> 1];
    const int X = s ? (i0 + VW == cx ? 0 : i0 + VW) : (i0 == 0 ? cx - 1 : i0 - 1);
    e = (((X + p) & 1) ? c1 : c0)[rb + (X >> 1)];
}

// Red-only trilinear correction, VW red cells per thread. The V-cycle's
// post-smoothing starts with a black half-sweep, which overwrites every black
// value without reading it, so correcting black cells would be a dead store;
// the result equals a correction of both colours followed by that sweep. The
// VW cells of a thread share their coarse rows: each of the four rows is read
// once (VW + 1 values).
template <typename T>
__device__ __forceinline__ void prolong_red_body(const T* __restrict__ cu0, const T* __restrict__ cu1, T* __restrict__ u0, int nx, int ny, int nz, Blk blk) {
    typedef typename VecOf<T>::type V;
    constexpr int VW = VecOf<T>::W;
    const int hx = nx >> 1, hv = hx / VW;
    const unsigned nv = (unsigned)hv * ny * nz;
    const unsigned idx = xcd_block(blk.b, blk.nb) * blockDim.x + threadIdx.x;
    if (idx >= nv) return;
    const int iv = idx % hv;
    const unsigned t = idx / hv;
    const int y = t % ny, z = t / ny;
    const int i0 = iv * VW;
    const int cx = nx >> 1, cy = ny >> 1, cz = nz >> 1;
    const int J0 = y >> 1, J1 = wrapi((y & 1) ? J0 + 1 : J0 - 1, cy);
    const int K0 = z >> 1, K1 = wrapi((z & 1) ? K0 + 1 : K0 - 1, cz);
    const int s0 = (y + z) & 1;  // red cell x = 2 (i0 + k) + s0: coarse I0 = i0 + k, I1 = I0 +/- 1
    const size_t row = ((size_t)z * ny + y) * hx;
    T m00[VW], m10[VW], m01[VW], m11[VW], e00, e10, e01, e11;
    coarse_row<T>(cu0, cu1, J0, K0, i0, s0, cx, cy, m00, e00);
    coarse_row<T>(cu0, cu1, J1, K0, i0, s0, cx, cy, m10, e10);
    coarse_row<T>(cu0, cu1, J0, K1, i0, s0, cx, cy, m01, e01);
    coarse_row<T>(cu0, cu1, J1, K1, i0, s0, cx, cy, m11, e11);
    V u = *reinterpret_cast<const V*>(u0 + row + i0);
#pragma unroll
    for (int k = 0; k < VW; ++k) {
        // the value at I1 = I0 + 1 (s0 = 1) or I0 - 1 (s0 = 0)
        const T n00 = s0 ? (k + 1 < VW ? m00[k + 1] : e00) : (k > 0 ? m00[k - 1] : e00);
        const T n10 = s0 ? (k + 1 < VW ? m10[k + 1] : e10) : (k > 0 ? m10[k - 1] : e10);
        const T n01 = s0 ? (k + 1 < VW ? m01[k + 1] : e01) : (k > 0 ? m01[k - 1] : e01);
        const T n11 = s0 ? (k + 1 < VW ? m11[k + 1] : e11) : (k > 0 ? m11[k - 1] : e11);
        u[k] = tri_add(u[k], m00[k], n00, m10[k], n10, m01[k], n01, m11[k], n11);
    }
    *reinterpret_cast<V*>(u0 + row + i0) = u;
}

template <typename T>
__global__ void __launch_bounds__(kMaxTuneBlock) k_prolong_red(const T* __restrict__ cu0, const T* __restrict__ cu1,
                                                        T* __restrict__ u0, int nx, int ny, int nz,
                                                        const Scalars* sc) {
    if (sc && sc->done) return;
    prolong_red_body<T>(cu0, cu1, u0, nx, ny, nz, Blk{blockIdx.x, gridDim.x});
}

template <typename T>
void launch_prolong(hipStream_t st, const T* cu0, const T* cu1, int coarse_natural, T* u0, T* u1, int nx, int ny,
                    int nz, const Scalars* sc, int bs) {
    constexpr int VW = VecOf<T>::W;
    const int hx = nx / 2;
    if (!coarse_natural && hx % VW == 0 && hx >= VW) {
        const unsigned nv = (unsigned)(hx / VW) * ny * nz;
        hipLaunchKernelGGL(k_prolong_red<T>, dim3(nblocks(nv, bs)), dim3(bs), 0, st, cu0, cu1, u0, nx, ny, nz, sc);
        return;
    }
    const unsigned nh = (unsigned)(nx / 2) * ny * nz;
    hipLaunchKernelGGL(k_prolong<T>, dim3(nblocks(nh, bs)), dim3(bs), 0, st, cu0, cu1, coarse_natural, u0, u1, nx, ny,
                       nz, sc);
}

// ---------------------------------------------------------------------------
// Temporally blocked forms for the small per-level levels, where a launch costs
// more than its bytes: one launch does the whole pre-smoothing, residual and
// restriction of a tile, one the whole correction and post-smoothing. A tile is
// 4 x 4 x 4 coarse cells (8^3 fine cells); it is computed in LDS from a halo that
// shrinks by one cell per half-sweep, so neighbouring tiles recompute their
// shared halo instead of synchronising. The arithmetic per cell is that of the
// per-step kernels, in the same order, so the results are bitwise identical.
constexpr int kTile = 8;             // fine tile edge
constexpr int kDownW = kTile + 10;   // pre-smoothing window: 5-cell halo
constexpr int kUpW = kTile + 8;      // post-smoothing window: 4-cell halo
constexpr int kUpCW = kTile / 2 + 6; // coarse window of the correction
constexpr int kResW = kTile + 2;     // residual window: 1-cell halo

inline size_t down_lds_bytes(size_t esz) { return esz * (2 * kDownW * kDownW * kDownW + kResW * kResW * kResW); }
inline size_t up_lds_bytes(size_t esz) { return esz * (2 * kUpW * kUpW * kUpW + kUpCW * kUpCW * kUpCW); }

// One half-sweep of the cells of colour `col` in the window cube [lo, hi)^3 of a
// W^3 LDS window; a cell's colour is (a + b + c + par) & 1 in window coordinates.
template <typename T, int W>
__device__ __forceinline__ void win_sweep(T* U, const T* F, int lo, int hi, int col, int par, T s, T inv_diag) {
    const int w = hi - lo, half = w >> 1, count = half * w * w;
    for (int j = threadIdx.x; j < count; j += blockDim.x) {
        const int i = j % half, t = j / half;
        const int b = lo + t % w, c = lo + t / w;
        const int a = lo + 2 * i + ((col + b + c + par - lo) & 1);
        const int k = (c * W + b) * W + a;
        U[k] = (F[k] + s * (((U[k - 1] + U[k + 1]) + (U[k - W] + U[k + W])) + (U[k - W * W] + U[k + W * W]))) *
               inv_diag;
    }
    __syncthreads();
}

// Pre-smoothing (black, red, black from the zero-guess red u0), red residual and
// restriction of the tile; writes the pre-smoothed red to `ured` (a separate
// array: neighbouring tiles still read u0 in their halos) and the coarse f and
// zero-guess red u of level l + 1 (split).
template <typename T>
__global__ void __launch_bounds__(kFinBlock) k_down(const T* __restrict__ u0, const T* __restrict__ f0,
                                                 const T* __restrict__ f1, T* __restrict__ ured, int nx, int ny, int nz,
                                                 T s, T inv_diag, T diag, T* __restrict__ cf0, T* __restrict__ cf1,
                                                 T* __restrict__ cu0, T inv_diag_c, const Scalars* sc) {
    if (sc && sc->done) return;
    constexpr int W = kDownW;
    extern __shared__ __align__(16) unsigned char smem[];
    T* U = reinterpret_cast<T*>(smem);
    T* F = U + W * W * W;
    T* R = F + W * W * W;
    const int hx = nx >> 1, cx = nx >> 1, cy = ny >> 1, cz = nz >> 1;
    const int tx = cx / 4, ty = cy / 4;
    const unsigned tile = xcd_block(blockIdx.x, gridDim.x);
    const int X0 = 4 * (int)(tile % tx), Y0 = 4 * (int)((tile / tx) % ty), Z0 = 4 * (int)(tile / (tx * ty));
    const int ox = 2 * X0 - 5, oy = 2 * Y0 - 5, oz = 2 * Z0 - 5;  // window origin (fine)
    for (int j = threadIdx.x; j < W * W * W; j += blockDim.x) {
        const int a = j % W, b = (j / W) % W, c = j / (W * W);
        const int x = wrapi(ox + a, nx), y = wrapi(oy + b, ny), z = wrapi(oz + c, nz);
        const size_t k = ((size_t)z * ny + y) * hx + (x >> 1);
        const int col = (x + y + z) & 1;
        F[j] = col ? f1[k] : f0[k];
        U[j] = col ? (T)0 : u0[k];
    }
    __syncthreads();
    // window colour parity: the origin offsets are odd on all three axes
    win_sweep<T, W>(U, F, 1, W - 1, 1, 1, s, inv_diag);
    win_sweep<T, W>(U, F, 2, W - 2, 0, 1, s, inv_diag);
    win_sweep<T, W>(U, F, 3, W - 3, 1, 1, s, inv_diag);
    constexpr int RW = kResW;
    for (int j = threadIdx.x; j < RW * RW * RW; j += blockDim.x) {
        const int a = 4 + j % RW, b = 4 + (j / RW) % RW, c = 4 + j / (RW * RW);
        const int k = (c * W + b) * W + a;
        R[j] = ((a + b + c + 1) & 1)
                   ? (T)0
                   : F[k] - (diag * U[k] -
                             s * (((U[k - 1] + U[k + 1]) + (U[k - W] + U[k + W])) + (U[k - W * W] + U[k + W * W])));
    }
    __syncthreads();
    // pre-smoothed red of the tile interior
    for (int j = threadIdx.x; j < kTile * kTile * kTile / 2; j += blockDim.x) {
        const int i = j % (kTile / 2), t = j / (kTile / 2);
        const int b = 5 + t % kTile, c = 5 + t / kTile;
        const int a = 5 + 2 * i + ((b + c) & 1);  // red: (a + b + c + 1) even
        const int x = ox + a, y = oy + b, z = oz + c;  // interior cells need no wrap
        ured[((size_t)z * ny + y) * hx + (x >> 1)] = U[(c * W + b) * W + a];
    }
    // restriction of the tile's 64 coarse cells (black residual zero): the four
    // z-planes of each coarse cell in parallel, then their weighted sum in order
    T* P = U;  // the sweep window is free now
    for (int j = threadIdx.x; j < 256; j += blockDim.x) {
        const int cell = j & 63, c = j >> 6;
        const int Xl = cell & 3, Yl = (cell >> 2) & 3, Zl = cell >> 4;
        const T w0 = (T)0.125, w1 = (T)0.375;
        T accb = 0;
#pragma unroll
        for (int b = 0; b < 4; ++b) {
            const T* row = R + ((2 * Zl + c) * RW + (2 * Yl + b)) * RW;  // fine y = 2Yl - 1 + b, +1 window shift
            const int p = (b + c) & 1;  // parity of the fine row: red cells at x = 2X - 1, 2X + 1 when 1
            const T ra = row[2 * Xl], rb = row[2 * Xl + 1], rc = row[2 * Xl + 2], rd = row[2 * Xl + 3];
            accb += (b == 0 || b == 3 ? w0 : w1) * restrict_row(w0, w1, p, p ? ra : (T)0, p ? rc : rb, p ? (T)0 : rd);
        }
        P[j] = accb;
    }
    __syncthreads();
    if (threadIdx.x < 64) {
        const int cell = threadIdx.x;
        const int Xl = cell & 3, Yl = (cell >> 2) & 3, Zl = cell >> 4;
        const T w0 = (T)0.125, w1 = (T)0.375;
        T acc = 0;
#pragma unroll
        for (int c = 0; c < 4; ++c) acc += (c == 0 || c == 3 ? w0 : w1) * P[c * 64 + cell];
        const int X = X0 + Xl, Y = Y0 + Yl, Z = Z0 + Zl;
        const size_t j = ((size_t)Z * cy + Y) * (cx >> 1) + (X >> 1);
        if ((X + Y + Z) & 1) {
            cf1[j] = acc;
        } else {
            cf0[j] = acc;
            cu0[j] = acc * inv_diag_c;
        }
    }
    (void)cz;
}

// Correction of the red cells from the coarse level (split), then
// post-smoothing (black, red, black, red); writes the tile's final u0 and u1.
template <typename T>
__global__ void __launch_bounds__(kFinBlock) k_up(const T* __restrict__ cu0, const T* __restrict__ cu1,
                                               const T* __restrict__ ured, const T* __restrict__ f0,
                                               const T* __restrict__ f1, T* __restrict__ u0, T* __restrict__ u1,
                                               int nx, int ny, int nz, T s, T inv_diag, const Scalars* sc) {
    if (sc && sc->done) return;
    constexpr int W = kUpW, CW = kUpCW;
    extern __shared__ __align__(16) unsigned char smem[];
    T* U = reinterpret_cast<T*>(smem);
    T* F = U + W * W * W;
    T* C = F + W * W * W;
    const int hx = nx >> 1, cx = nx >> 1, cy = ny >> 1, cz = nz >> 1;
    const int tx = cx / 4, ty = cy / 4;
    const unsigned tile = xcd_block(blockIdx.x, gridDim.x);
    const int X0 = 4 * (int)(tile % tx), Y0 = 4 * (int)((tile / tx) % ty), Z0 = 4 * (int)(tile / (tx * ty));
    const int ox = 2 * X0 - 4, oy = 2 * Y0 - 4, oz = 2 * Z0 - 4;  // window origin (fine)
    const int cox = X0 - 3, coy = Y0 - 3, coz = Z0 - 3;          // coarse window origin
    for (int j = threadIdx.x; j < CW * CW * CW; j += blockDim.x) {
        const int a = j % CW, b = (j / CW) % CW, c = j / (CW * CW);
        C[j] = coarse_at(cu0, cu1, 0, wrapi(cox + a, cx), wrapi(coy + b, cy), wrapi(coz + c, cz), cx, cy);
    }
    __syncthreads();
    for (int j = threadIdx.x; j < W * W * W; j += blockDim.x) {
        const int a = j % W, b = (j / W) % W, c = j / (W * W);
        const int xu = ox + a, yu = oy + b, zu = oz + c;  // unwrapped fine coordinates
        const int x = wrapi(xu, nx), y = wrapi(yu, ny), z = wrapi(zu, nz);
        const size_t k = ((size_t)z * ny + y) * hx + (x >> 1);
        const int col = (x + y + z) & 1;
        F[j] = col ? f1[k] : f0[k];
        if (col) {
            U[j] = (T)0;
        } else {
            // trilinear weights 3/4 (own coarse cell) and 1/4 (the neighbour on the cell's side)
            const int I0 = (xu >> 1) - cox, I1 = (xu & 1) ? I0 + 1 : I0 - 1;
            const int J0 = (yu >> 1) - coy, J1 = (yu & 1) ? J0 + 1 : J0 - 1;
            const int K0 = (zu >> 1) - coz, K1 = (zu & 1) ? K0 + 1 : K0 - 1;
            const T* c00 = C + (K0 * CW + J0) * CW;
            const T* c10 = C + (K0 * CW + J1) * CW;
            const T* c01 = C + (K1 * CW + J0) * CW;
            const T* c11 = C + (K1 * CW + J1) * CW;
            U[j] = tri_add(ured[k], c00[I0], c00[I1], c10[I0], c10[I1], c01[I0], c01[I1], c11[I0], c11[I1]);
        }
    }
    __syncthreads();
    // window colour parity: the origin offsets are even
    win_sweep<T, W>(U, F, 1, W - 1, 1, 0, s, inv_diag);
    win_sweep<T, W>(U, F, 2, W - 2, 0, 0, s, inv_diag);
    win_sweep<T, W>(U, F, 3, W - 3, 1, 0, s, inv_diag);
    win_sweep<T, W>(U, F, 4, W - 4, 0, 0, s, inv_diag);
    for (int j = threadIdx.x; j < kTile * kTile * kTile; j += blockDim.x) {
        const int a = 4 + j % kTile, b = 4 + (j / kTile) % kTile, c = 4 + j / (kTile * kTile);
        const int x = ox + a, y = oy + b, z = oz + c;
        const size_t k = ((size_t)z * ny + y) * hx + (x >> 1);
        const T v = U[(c * W + b) * W + a];
        if ((x + y + z) & 1) u1[k] = v;
        else u0[k] = v;
    }
}

template <typename T>
void launch_down(hipStream_t st, const T* u0, const T* f0, const T* f1, T* ured, int nx, int ny, int nz, double s,
                 double diag, T* cf0, T* cf1, T* cu0, double inv_diag_c, const Scalars* sc) {
    const unsigned nt = (unsigned)(nx / 8) * (ny / 8) * (nz / 8);
    const unsigned bs = nt <= 512 ? kFinBlock : kBlock;  // few tiles: more threads per tile
    hipLaunchKernelGGL(k_down<T>, dim3(nt), dim3(bs), down_lds_bytes(sizeof(T)), st, u0, f0, f1, ured, nx, ny, nz,
                       (T)s, (T)(1.0 / diag), (T)diag, cf0, cf1, cu0, (T)inv_diag_c, sc);
}

template <typename T>
void launch_up(hipStream_t st, const T* cu0, const T* cu1, const T* ured, const T* f0, const T* f1, T* u0, T* u1,
               int nx, int ny, int nz, double s, double diag, const Scalars* sc) {
    const unsigned nt = (unsigned)(nx / 8) * (ny / 8) * (nz / 8);
    const unsigned bs = nt <= 512 ? kFinBlock : kBlock;  // few tiles: more threads per tile
    hipLaunchKernelGGL(k_up<T>, dim3(nt), dim3(bs), up_lds_bytes(sizeof(T)), st, cu0, cu1, ured, f0, f1, u0, u1,
                       nx, ny, nz, (T)s, (T)(1.0 / diag), sc);
}

template <typename T>
hipError_t blocked_set_lds() {
    hipError_t e = hipFuncSetAttribute((const void*)k_down<T>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                       (int)down_lds_bytes(sizeof(T)));
    if (e != hipSuccess) return e;
    return hipFuncSetAttribute((const void*)k_up<T>, hipFuncAttributeMaxDynamicSharedMemorySize,
                               (int)up_lds_bytes(sizeof(T)));
}

// ---------------------------------------------------------------------------
// Coarsest grid: u = C f with C the dense FP64 (pseudo-)inverse, m <= 512.
template <typename T>
__global__ void __launch_bounds__(kMaxCoarse) k_coarse(const T* __restrict__ f, T* __restrict__ u,
                                                       const double* __restrict__ cinv, int m, const Scalars* sc) {
    if (sc && sc->done) return;
    __shared__ double fs[kMaxCoarse];
    for (int j = threadIdx.x; j < m; j += blockDim.x) fs[j] = (double)f[j];
    __syncthreads();
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6, nw = blockDim.x >> 6;
    for (int i = wv; i < m; i += nw) {
        const double* row = cinv + (size_t)i * m;
        double acc = 0.0;
        for (int j = lane; j < m; j += 64) acc += row[j] * fs[j];
        acc = wave_sum(acc);
        if (lane == 0) u[i] = (T)acc;
    }
}

template <typename T>
void launch_coarse(hipStream_t st, const T* f, T* u, const double* cinv, int m, const Scalars* sc) {
    hipLaunchKernelGGL(k_coarse<T>, dim3(1), dim3(kMaxCoarse), 0, st, f, u, cinv, m, sc);
}

// ---------------------------------------------------------------------------
// Coarse tail: the whole V-cycle below level t in one work-group with every
// level in LDS (natural layout [z][y][x]). It performs exactly the operations
// of the per-level kernels, in the same order and with the same summation
// order, so it is interchangeable with them: zero initial guess, R B R B
// pre-smoothing, residual, full weighting, coarse dense solve, trilinear
// correction, B R B R post-smoothing.
// Thread-strided loops over each level's cells; cell coordinates are decoded
// on the fly (shifts and masks for power-of-two dimensions), so no per-thread
// cell tables are kept live across the barriers.
__device__ __forceinline__ bool tail_pow2(int a) { return (a & (a - 1)) == 0; }

// j -> (a, b, c) for row-major dims (na, nb, *).
__device__ __forceinline__ void tail_decode(int j, int na, int nb, bool p2, int la, int lab, int& a, int& b, int& c) {
    if (p2) {
        a = j & (na - 1);
        b = (j >> la) & (nb - 1);
        c = j >> lab;
    } else {
        a = j % na;
        const int t = j / na;
        b = t % nb;
        c = t / nb;
    }
}

// Decoder of one (na, nb) plane shape: uniform across the work-group.
struct TailDec {
    int na, nb, la, lab;
    bool p2;
    __device__ __forceinline__ TailDec(int a, int b) : na(a), nb(b) {
        p2 = tail_pow2(a) && tail_pow2(b);
        la = __ffs(a) - 1;
        lab = la + __ffs(b) - 1;
    }
    __device__ __forceinline__ void operator()(int j, int& x, int& y, int& z) const {
        tail_decode(j, na, nb, p2, la, lab, x, y, z);
    }
};

template <typename T>
__device__ __forceinline__ T tail_nb(const T* u, int x, int y, int z, int nx, int ny, int nz) {
    const int row = (z * ny + y) * nx;
    const T a = u[row + wrapi(x - 1, nx)] + u[row + wrapi(x + 1, nx)];
    const T b = u[(z * ny + wrapi(y - 1, ny)) * nx + x] + u[(z * ny + wrapi(y + 1, ny)) * nx + x];
    const T c = u[(wrapi(z - 1, nz) * ny + y) * nx + x] + u[(wrapi(z + 1, nz) * ny + y) * nx + x];
    return (a + b) + c;
}

// One half-sweep of colour `color` (red: x + y + z even) in LDS.
template <typename T>
__device__ __forceinline__ void tail_gs(T* u, const T* f, int nx, int ny, int nz, int color, T s, T inv_diag) {
    const int hx = nx >> 1, nh = hx * ny * nz;
    const TailDec dec(hx, ny);
    for (int j = threadIdx.x; j < nh; j += blockDim.x) {
        int i, y, z;
        dec(j, i, y, z);
        const int x = 2 * i + ((y + z + color) & 1);
        const int k = (z * ny + y) * nx + x;
        u[k] = (f[k] + s * tail_nb(u, x, y, z, nx, ny, nz)) * inv_diag;
    }
    __syncthreads();
}

// Coarse tail: the whole V-cycle below level t in one work-group with every
// level in LDS (natural layout [z][y][x]). It performs exactly the operations
// of the per-level kernels, in the same order and with the same summation
// order, so it is interchangeable with them: zero initial guess, R B R B
// pre-smoothing, residual, full weighting, coarse dense solve, trilinear
// correction, B R B R post-smoothing.
template <typename T>
__device__ __forceinline__ void tail_body(const T* __restrict__ f0g, const T* __restrict__ f1g, T* __restrict__ u0g,
                                          T* __restrict__ u1g, const TailDesc& d, const double* __restrict__ cinv) {
    extern __shared__ __align__(16) unsigned char smem[];
#define TAIL_U(l) reinterpret_cast<T*>(smem + d.off_u[l])
#define TAIL_F(l) reinterpret_cast<T*>(smem + d.off_f[l])
#define TAIL_R(l) reinterpret_cast<T*>(smem + d.off_r[l])
    const int L = d.nlev - 1;  // coarsest, natural, m cells
    {
        // split (red, black) global arrays -> natural LDS level 0
        const int nx = d.nx[0], ny = d.ny[0], hx = nx >> 1, nh = hx * ny * d.nz[0];
        const TailDec dec(hx, ny);
        T* F0 = TAIL_F(0);
        for (int j = threadIdx.x; j < nh; j += blockDim.x) {
            int i, y, z;
            dec(j, i, y, z);
            const int row = (z * ny + y) * nx, par = (y + z) & 1;
            F0[row + 2 * i + par] = f0g[j];
            F0[row + 2 * i + (par ^ 1)] = f1g[j];
        }
    }
    __syncthreads();
    for (int l = 0; l < L; ++l) {
        const int nx = d.nx[l], ny = d.ny[l], nz = d.nz[l], n = nx * ny * nz;
        T* U = TAIL_U(l);
        T* F = TAIL_F(l);
        T* R = TAIL_R(l);
        const T s = (T)d.s[l], idg = (T)d.inv_diag[l], dg = (T)d.diag[l];
        for (int j = threadIdx.x; j < n; j += blockDim.x) U[j] = (T)0;
        __syncthreads();
        tail_gs(U, F, nx, ny, nz, 0, s, idg);
        tail_gs(U, F, nx, ny, nz, 1, s, idg);
        tail_gs(U, F, nx, ny, nz, 0, s, idg);
        tail_gs(U, F, nx, ny, nz, 1, s, idg);
        {
            const TailDec dec(nx, ny);
            for (int j = threadIdx.x; j < n; j += blockDim.x) {
                int x, y, z;
                dec(j, x, y, z);
                R[j] = ((x + y + z) & 1) ? (T)0 : F[j] - (dg * U[j] - s * tail_nb(U, x, y, z, nx, ny, nz));
            }
        }
        __syncthreads();
        const int cx = nx >> 1, cy = ny >> 1, nc = cx * cy * (nz >> 1);
        T* Fc = TAIL_F(l + 1);
        const T w0 = (T)0.125, w1 = (T)0.375;
        const TailDec cdec(cx, cy);
        for (int j = threadIdx.x; j < nc; j += blockDim.x) {
            int X, Y, Z;
            cdec(j, X, Y, Z);
            const int x0 = wrapi(2 * X - 1, nx), x1 = 2 * X, x2 = 2 * X + 1, x3 = wrapi(2 * X + 2, nx);
            T acc = 0;
#pragma unroll
            for (int c = 0; c < 4; ++c) {
                const int z = wrapi(2 * Z - 1 + c, nz);
                T accb = 0;
#pragma unroll
                for (int b = 0; b < 4; ++b) {
                    const T* rr = R + (z * ny + wrapi(2 * Y - 1 + b, ny)) * nx;
                    const T acca = ((w0 * rr[x0] + w1 * rr[x1]) + w1 * rr[x2]) + w0 * rr[x3];
                    accb += (b == 0 || b == 3 ? w0 : w1) * acca;
                }
                acc += (c == 0 || c == 3 ? w0 : w1) * accb;
            }
            Fc[j] = acc;
        }
        __syncthreads();
    }
    {
        // one wave per row of the dense inverse: coalesced loads, wave reduction
        const T* Fl = TAIL_F(L);
        T* Ul = TAIL_U(L);
        const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6, nw = blockDim.x >> 6;
        for (int i = wv; i < d.m; i += nw) {
            const double* row = cinv + (size_t)i * d.m;
            double acc = 0.0;
            for (int j = lane; j < d.m; j += 64) acc += row[j] * (double)Fl[j];
            acc = wave_sum(acc);
            if (lane == 0) Ul[i] = (T)acc;
        }
    }
    __syncthreads();
    for (int l = L - 1; l >= 0; --l) {
        const int nx = d.nx[l], ny = d.ny[l], nz = d.nz[l], n = nx * ny * nz;
        const int cx = nx >> 1, cy = ny >> 1, cz = nz >> 1;
        const T* C = TAIL_U(l + 1);
        T* U = TAIL_U(l);
        const T* F = TAIL_F(l);
        const TailDec dec(nx, ny);
        for (int j = threadIdx.x; j < n; j += blockDim.x) {
            int x, y, z;
            dec(j, x, y, z);
            const int I0 = x >> 1, I1 = wrapi((x & 1) ? I0 + 1 : I0 - 1, cx);
            const int J0 = y >> 1, J1 = wrapi((y & 1) ? J0 + 1 : J0 - 1, cy);
            const int K0 = z >> 1, K1 = wrapi((z & 1) ? K0 + 1 : K0 - 1, cz);
            const T* c00 = C + (K0 * cy + J0) * cx;
            const T* c10 = C + (K0 * cy + J1) * cx;
            const T* c01 = C + (K1 * cy + J0) * cx;
            const T* c11 = C + (K1 * cy + J1) * cx;
            U[j] = tri_add(U[j], c00[I0], c00[I1], c10[I0], c10[I1], c01[I0], c01[I1], c11[I0], c11[I1]);
        }
        __syncthreads();
        const T s = (T)d.s[l], idg = (T)d.inv_diag[l];
        tail_gs(U, F, nx, ny, nz, 1, s, idg);
        tail_gs(U, F, nx, ny, nz, 0, s, idg);
        tail_gs(U, F, nx, ny, nz, 1, s, idg);
        tail_gs(U, F, nx, ny, nz, 0, s, idg);
    }
    {
        const int nx = d.nx[0], ny = d.ny[0], hx = nx >> 1, nh = hx * ny * d.nz[0];
        const TailDec dec(hx, ny);
        const T* U0 = TAIL_U(0);
        for (int j = threadIdx.x; j < nh; j += blockDim.x) {
            int i, y, z;
            dec(j, i, y, z);
            const int row = (z * ny + y) * nx, par = (y + z) & 1;
            u0g[j] = U0[row + 2 * i + par];
            u1g[j] = U0[row + 2 * i + (par ^ 1)];
        }
    }
#undef TAIL_U
#undef TAIL_F
#undef TAIL_R
}

template <typename T>
__global__ void __launch_bounds__(kFinBlock) k_tail(const T* __restrict__ f0g, const T* __restrict__ f1g,
                                                    T* __restrict__ u0g, T* __restrict__ u1g, TailDesc d,
                                                    const double* __restrict__ cinv, const Scalars* sc) {
    if (sc && sc->done) return;
    tail_body<T>(f0g, f1g, u0g, u1g, d, cinv);
}

template <typename T>
void launch_tail(hipStream_t st, const T* f0, const T* f1, T* u0, T* u1, const TailDesc& d, const double* cinv,
                 const Scalars* sc) {
    hipLaunchKernelGGL(k_tail<T>, dim3(1), dim3(kFinBlock), d.lds_bytes, st, f0, f1, u0, u1, d, cinv, sc);
}

template <typename T>
hipError_t tail_set_lds(size_t bytes) {
    return hipFuncSetAttribute((const void*)k_tail<T>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
}

// ---------------------------------------------------------------------------
// Batched forms: one launch covers one level of every instance in the table
// (the same bodies as the solo kernels, so results are bitwise the same).
template <typename T>
__global__ void __launch_bounds__(kBlock) kb_gs(const InstDev* inst, const int* gate, const BatchTab* tab, int l, int color) {
    const BatchEntry* ent = tab_entries(tab);
    for (unsigned g = blockIdx.x; g < tab->total; g += gridDim.x) {
        Blk blk;
        const InstDev* I = batch_slot(inst, gate, ent, tab->n, g, blk);
        if (!I) continue;
        T* const* a = reinterpret_cast<T* const*>(I->lv[l]);
        const int c = color;
        gs_vec_body<T>(a[c ? 1 : 0], a[c ? 0 : 1], a[c ? 3 : 2], I->lnx[l] >> 1, I->lny[l], I->lnz[l], c,
                       (T)I->ls[l], (T)(1.0 / I->ldiag[l]), blk);
    }
}

template <typename T>
__global__ void __launch_bounds__(kBlock) kb_gs_dots(const InstDev* inst, const int* gate, const BatchTab* tab) {
    const BatchEntry* ent = tab_entries(tab);
    for (unsigned g = blockIdx.x; g < tab->total; g += gridDim.x) {
        Blk blk;
        const InstDev* I = batch_slot(inst, gate, ent, tab->n, g, blk);
        if (!I) continue;
        T* const* a = reinterpret_cast<T* const*>(I->lv[0]);
        gs_vec_dots_body<T>(a[0], a[1], a[2], I->lnx[0] >> 1, I->lny[0], I->lnz[0], (T)I->ls[0],
                            (T)(1.0 / I->ldiag[0]), I->r, I->q, I->part, blk);
        __syncthreads();  // partial-sum scratch is reused by the next virtual block
    }
}

template <typename T>
__global__ void __launch_bounds__(kBlock) kb_resid(const InstDev* inst, const int* gate, const BatchTab* tab, int l) {
    const BatchEntry* ent = tab_entries(tab);
    for (unsigned g = blockIdx.x; g < tab->total; g += gridDim.x) {
        Blk blk;
        const InstDev* I = batch_slot(inst, gate, ent, tab->n, g, blk);
        if (!I) continue;
        T* const* a = reinterpret_cast<T* const*>(I->lv[l]);
        resid_vec_body<T>(a[0], a[1], a[2], a[4], I->lnx[l] >> 1, I->lny[l], I->lnz[l], (T)I->ls[l],
                          (T)I->ldiag[l], blk);
    }
}

template <typename T>
__global__ void __launch_bounds__(kBlock) kb_restrict(const InstDev* inst, const int* gate, const BatchTab* tab, int l) {
    const BatchEntry* ent = tab_entries(tab);
    for (unsigned g = blockIdx.x; g < tab->total; g += gridDim.x) {
        Blk blk;
        const InstDev* I = batch_slot(inst, gate, ent, tab->n, g, blk);
        if (!I) continue;
        T* const* a = reinterpret_cast<T* const*>(I->lv[l]);
        T* const* c = reinterpret_cast<T* const*>(I->lv[l + 1]);
        restrict4_body<T>(a[4], I->lnx[l], I->lny[l], I->lnz[l], c[2], c[3], c[0], 0, (T)(1.0 / I->ldiag[l + 1]),
                          blk);
    }
}

template <typename T>
__global__ void __launch_bounds__(kBlock) kb_prolong(const InstDev* inst, const int* gate, const BatchTab* tab, int l) {
    const BatchEntry* ent = tab_entries(tab);
    for (unsigned g = blockIdx.x; g < tab->total; g += gridDim.x) {
        Blk blk;
        const InstDev* I = batch_slot(inst, gate, ent, tab->n, g, blk);
        if (!I) continue;
        T* const* a = reinterpret_cast<T* const*>(I->lv[l]);
        T* const* c = reinterpret_cast<T* const*>(I->lv[l + 1]);
        prolong_red_body<T>(c[0], c[1], a[0], I->lnx[l], I->lny[l], I->lnz[l], blk);
    }
}

// One work-group per instance: the coarse tail from the instance's level t.
template <typename T>
__global__ void __launch_bounds__(kFinBlock) kb_tail(const InstDev* inst, const int* gate, int ninst) {
    const int i = blockIdx.x;
    if (i >= ninst || !gate[i]) return;
    const InstDev* I = inst + i;
    if (I->sc->done) return;
    T* const* a = reinterpret_cast<T* const*>(I->lv[I->t]);
    tail_body<T>(a[2], a[3], a[0], a[1], I->tail, I->cinv);
}

template <typename T>
void launchb_mg(hipStream_t st, int what, const InstDev* inst, const int* gate, const BatchTab* tab, unsigned grid,
                int l, int color, unsigned lds) {
    const dim3 g(grid), b(kBlock);
    switch (what) {
        case BMG_GS: hipLaunchKernelGGL(kb_gs<T>, g, b, 0, st, inst, gate, tab, l, color); break;
        case BMG_GS_DOTS: hipLaunchKernelGGL(kb_gs_dots<T>, g, b, 0, st, inst, gate, tab); break;
        case BMG_RESID: hipLaunchKernelGGL(kb_resid<T>, g, b, 0, st, inst, gate, tab, l); break;
        case BMG_RESTRICT: hipLaunchKernelGGL(kb_restrict<T>, g, b, 0, st, inst, gate, tab, l); break;
        case BMG_PROLONG: hipLaunchKernelGGL(kb_prolong<T>, g, b, 0, st, inst, gate, tab, l); break;
        default: hipLaunchKernelGGL(kb_tail<T>, dim3(grid), dim3(kFinBlock), lds, st, inst, gate, (int)grid);
    }
}

template <typename T>
hipError_t tail_set_lds_batched(size_t bytes) {
    return hipFuncSetAttribute((const void*)kb_tail<T>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
}

#define BRD_INST(T)                                                                                                \
    template void launch_enter<T>(hipStream_t, const double*, T*, T*, T*, int, int, int, double, const Scalars*);  \
    template void launch_resid_enter<T>(hipStream_t, const double*, const T*, const T*, T*, T*, T*, int, int, int, \
                                        double, double, double);                                                    \
    template void launch_gs<T>(hipStream_t, T*, const T*, const T*, int, int, int, int, double, double,            \
                               const Scalars*, int);                                                               \
    template bool launch_gs_from_f<T>(hipStream_t, T*, const T*, const T*, int, int, int, int, double, double,     \
                                      const Scalars*, int);                                                        \
    template void launch_resid_red<T>(hipStream_t, const T*, const T*, const T*, T*, int, int, int, double, double, \
                                      const Scalars*, int);                                                         \
    template void launch_restrict<T>(hipStream_t, const T*, int, int, int, T*, T*, T*, int, double, const Scalars*, \
                                     int);                                                                          \
    template void launch_prolong<T>(hipStream_t, const T*, const T*, int, T*, T*, int, int, int, const Scalars*,    \
                                    int);                                                                           \
    template unsigned launch_gs_dots<T>(hipStream_t, T*, const T*, const T*, int, int, int, double, double,         \
                                        const double*, const double*, double*, const Scalars*, int);                \
    template void launch_coarse<T>(hipStream_t, const T*, T*, const double*, int, const Scalars*);             \
    template void launch_tail<T>(hipStream_t, const T*, const T*, T*, T*, const TailDesc&, const double*,         \
                                 const Scalars*);                                                                   \
    template hipError_t tail_set_lds<T>(size_t);                                                                   \
    template void launch_down<T>(hipStream_t, const T*, const T*, const T*, T*, int, int, int, double, double, T*, T*, \
                                 T*, double, const Scalars*);                                                      \
    template void launch_up<T>(hipStream_t, const T*, const T*, const T*, const T*, const T*, T*, T*, int, int, int,  \
                               double, double, const Scalars*);                                                    \
    template hipError_t blocked_set_lds<T>();                                                                      \
    template void launchb_mg<T>(hipStream_t, int, const InstDev*, const int*, const BatchTab*, unsigned, int, int,   \
                                unsigned);                                                                         \
    template hipError_t tail_set_lds_batched<T>(size_t);

BRD_INST(float)
BRD_INST(double)

}  // namespace brd
