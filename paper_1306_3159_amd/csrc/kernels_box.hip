// Multigrid kernels for alpha I - D L_0 in a box whose faces hold a fixed value.
//
// The single-blob tests of arXiv:1306.3159 (Sec. IV.C, eq. c_r_approx) keep the
// concentration at c_inf on the faces of a cubic box. The solves work on the
// homogeneous part u = c - c_inf, so L_0 is the cell-centred 7-point Laplacian
// whose ghost beyond a face is -u of the boundary cell (the face value is the
// mean of the two). A cell touching f faces then has the diagonal
// alpha + s (6 + f), s = D / h^2, and no neighbour term across those faces.
//
// The V-cycle is the periodic one (V(2,2) red-black Gauss-Seidel, red-only
// residual and correction, R = P^T / 8, rediscretised coarse operators) with
// the box operator on every level and the ghost -u in the transfers: a fine
// boundary cell interpolates (3/4 - 1/4) of its coarse parent, which is linear
// interpolation to the zero face value, and the restriction is the transpose.
//
// Layout: the red/black split layout of the periodic levels (cell (x, y, z) of
// colour c = (x+y+z)&1 at index x/2 of row (y, z) of array c), one cell per
// thread; the coarsest level is natural.
#include "launch.hpp"

namespace brd {

namespace {

// Decode a split index into (half-index i, row y, z).
__device__ __forceinline__ void split_pos(unsigned idx, int hx, int ny, int& i, int& y, int& z) {
    i = idx % hx;
    const unsigned t = idx / hx;
    y = t % ny;
    z = t / ny;
}

// Sum of the in-box neighbours of the cell at x = 2i + so in row (y, z), read
// from the other colour's array uo (absent neighbours add nothing).
template <typename T>
__device__ __forceinline__ T box_nb_sum(const T* __restrict__ uo, int i, int y, int z, int nx, int ny, int nz,
                                        int so) {
    const int hx = nx >> 1;
    const int x = 2 * i + so;
    const size_t row = ((size_t)z * ny + y) * hx;
    const size_t plane = (size_t)ny * hx;
    const T xm = x > 0 ? uo[row + i - 1 + so] : (T)0;
    const T xp = x + 1 < nx ? uo[row + i + so] : (T)0;
    const T ym = y > 0 ? uo[row - hx + i] : (T)0;
    const T yp = y + 1 < ny ? uo[row + hx + i] : (T)0;
    const T zm = z > 0 ? uo[row - plane + i] : (T)0;
    const T zp = z + 1 < nz ? uo[row + plane + i] : (T)0;
    return ((xm + xp) + (ym + yp)) + (zm + zp);
}

// 16-byte vectors of the split rows: 4 FP32 or 2 FP64 cells per thread.
template <typename T>
struct BoxVec;
template <>
struct BoxVec<float> {
    typedef float type __attribute__((ext_vector_type(4)));
    static constexpr int W = 4;
};
template <>
struct BoxVec<double> {
    typedef double type __attribute__((ext_vector_type(2)));
    static constexpr int W = 2;
};

// Row vector i0 .. i0+VW-1 of colour c (x = 2i + so) and the in-box neighbour sums of
// its cells from the other colour's array uo. An x-neighbour beyond a face exists only
// for the first cell of a row (so = 0, x = 0) and the last one (so = 1, x = nx - 1);
// y/z neighbour rows beyond a face contribute nothing.
template <typename T>
__device__ __forceinline__ typename BoxVec<T>::type box_nb_vec(const T* __restrict__ uo, int i0, int y, int z, int nx,
                                                               int ny, int nz, int so) {
    typedef typename BoxVec<T>::type V;
    constexpr int VW = BoxVec<T>::W;
    const int hx = nx >> 1;
    const size_t row = ((size_t)z * ny + y) * hx;
    const size_t plane = (size_t)ny * hx;
    const T* orow = uo + row;
    const V o = *reinterpret_cast<const V*>(orow + i0);
    const T edge = so ? (i0 + VW < hx ? orow[i0 + VW] : (T)0) : (i0 > 0 ? orow[i0 - 1] : (T)0);
    const V zero = (V)(T)0;
    const V ym = y > 0 ? *reinterpret_cast<const V*>(orow - hx + i0) : zero;
    const V yp = y + 1 < ny ? *reinterpret_cast<const V*>(orow + hx + i0) : zero;
    const V zm = z > 0 ? *reinterpret_cast<const V*>(orow - plane + i0) : zero;
    const V zp = z + 1 < nz ? *reinterpret_cast<const V*>(orow + plane + i0) : zero;
    V nb;
#pragma unroll
    for (int k = 0; k < VW; ++k) {
        const T left = so ? o[k] : (k ? o[k - 1] : edge);
        const T right = so ? (k + 1 < VW ? o[k + 1] : edge) : o[k];
        nb[k] = ((left + right) + (ym[k] + yp[k])) + (zm[k] + zp[k]);
    }
    return nb;
}

// Face count of cell k of the row vector: the y/z faces of the row plus x = 0 (first
// cell, so = 0) or x = nx - 1 (last cell, so = 1).
template <int VW>
__device__ __forceinline__ int box_faces_vec(int k, int i0, int hx, int so, int fyz) {
    return fyz + ((so == 0 && i0 == 0 && k == 0) || (so == 1 && i0 + VW == hx && k == VW - 1) ? 1 : 0);
}

}  // namespace

// Fine-level entry: f = r (FP64 natural -> T split) and the first red
// half-sweep from a zero guess, u_red = f_red / diag(cell).
template <typename T>
__global__ void __launch_bounds__(kBlock) k_enter_box(const double* __restrict__ r, T* __restrict__ f0,
                                                      T* __restrict__ f1, T* __restrict__ u0, int nx, int ny, int nz,
                                                      BoxCoef inv, const Scalars* sc) {
    if (sc && sc->done) return;
    const int hx = nx >> 1;
    const unsigned nh = (unsigned)hx * ny * nz;
    const unsigned idx = xcd_block(blockIdx.x, gridDim.x) * blockDim.x + threadIdx.x;
    if (idx >= nh) return;
    int i, y, z;
    split_pos(idx, hx, ny, i, y, z);
    const int s0 = (y + z) & 1;  // x offset of the red cell in this row
    const size_t rowN = ((size_t)z * ny + y) * nx;
    const double fr = r[rowN + 2 * i + s0];
    const double fb = r[rowN + 2 * i + (s0 ^ 1)];
    f0[idx] = (T)fr;
    f1[idx] = (T)fb;
    u0[idx] = (T)((T)fr * (T)inv.v[box_faces(2 * i + s0, y, z, nx, ny, nz)]);
}

template <typename T>
void launch_enter_box(hipStream_t st, const double* r, T* f0, T* f1, T* u0, int nx, int ny, int nz,
                      const BoxCoef& inv, const Scalars* sc) {
    const unsigned nh = (unsigned)(nx / 2) * ny * nz;
    hipLaunchKernelGGL(k_enter_box<T>, dim3(nblocks(nh)), dim3(kBlock), 0, st, r, f0, f1, u0, nx, ny, nz, inv, sc);
}

// Gauss-Seidel half-sweep on colour `color`: u_c = (f_c + s * sum of in-box neighbours) / diag(cell).
template <typename T>
__global__ void __launch_bounds__(kBlock) k_gs_box(T* __restrict__ uc, const T* __restrict__ uo,
                                                   const T* __restrict__ fc, int nx, int ny, int nz, int color, T s,
                                                   BoxCoef inv, const Scalars* sc) {
    if (sc && sc->done) return;
    const int hx = nx >> 1;
    const unsigned nh = (unsigned)hx * ny * nz;
    const unsigned idx = xcd_block(blockIdx.x, gridDim.x) * blockDim.x + threadIdx.x;
    if (idx >= nh) return;
    int i, y, z;
    split_pos(idx, hx, ny, i, y, z);
    const int so = ((y + z) & 1) ^ color;
    const T nb = box_nb_sum(uo, i, y, z, nx, ny, nz, so);
    uc[idx] = (fc[idx] + s * nb) * (T)inv.v[box_faces(2 * i + so, y, z, nx, ny, nz)];
}

// Vector form: VW cells of a split row per thread (needs (nx/2) % VW == 0).
template <typename T>
__global__ void __launch_bounds__(kBlock) k_gs_box_vec(T* __restrict__ uc, const T* __restrict__ uo,
                                                       const T* __restrict__ fc, int nx, int ny, int nz, int color,
                                                       T s, BoxCoef inv, const Scalars* sc) {
    if (sc && sc->done) return;
    typedef typename BoxVec<T>::type V;
    constexpr int VW = BoxVec<T>::W;
    const int hx = nx >> 1, hv = hx / VW;
    const unsigned nv = (unsigned)hv * ny * nz;
    const unsigned idx = xcd_block(blockIdx.x, gridDim.x) * blockDim.x + threadIdx.x;
    if (idx >= nv) return;
    int iv, y, z;
    split_pos(idx, hv, ny, iv, y, z);
    const int i0 = iv * VW;
    const int so = ((y + z) & 1) ^ color;
    const V nb = box_nb_vec<T>(uo, i0, y, z, nx, ny, nz, so);
    const size_t row = ((size_t)z * ny + y) * hx;
    const V f = *reinterpret_cast<const V*>(fc + row + i0);
    const int fyz = (y == 0) + (y + 1 == ny) + (z == 0) + (z + 1 == nz);
    V out;
#pragma unroll
    for (int k = 0; k < VW; ++k)
        out[k] = (f[k] + s * nb[k]) * (T)inv.v[box_faces_vec<VW>(k, i0, hx, so, fyz)];
    *reinterpret_cast<V*>(uc + row + i0) = out;
}

template <typename T>
void launch_gs_box(hipStream_t st, T* uc, const T* uo, const T* fc, int nx, int ny, int nz, int color, double s,
                   const BoxCoef& inv, const Scalars* sc) {
    constexpr int VW = BoxVec<T>::W;
    if ((nx / 2) % VW == 0) {
        const unsigned nv = (unsigned)(nx / 2 / VW) * ny * nz;
        hipLaunchKernelGGL(k_gs_box_vec<T>, dim3(nblocks(nv)), dim3(kBlock), 0, st, uc, uo, fc, nx, ny, nz, color,
                           (T)s, inv, sc);
        return;
    }
    const unsigned nh = (unsigned)(nx / 2) * ny * nz;
    hipLaunchKernelGGL(k_gs_box<T>, dim3(nblocks(nh)), dim3(kBlock), 0, st, uc, uo, fc, nx, ny, nz, color, (T)s, inv,
                       sc);
}

// Red residual after pre-smoothing (the closing black half-sweep leaves the
// black residual zero): r0 = f0 - (diag(cell) u0 - s * sum of black neighbours).
template <typename T>
__global__ void __launch_bounds__(kBlock) k_resid_box(const T* __restrict__ u0, const T* __restrict__ u1,
                                                      const T* __restrict__ f0, T* __restrict__ r0, int nx, int ny,
                                                      int nz, T s, BoxCoef diag, const Scalars* sc) {
    if (sc && sc->done) return;
    const int hx = nx >> 1;
    const unsigned nh = (unsigned)hx * ny * nz;
    const unsigned idx = xcd_block(blockIdx.x, gridDim.x) * blockDim.x + threadIdx.x;
    if (idx >= nh) return;
    int i, y, z;
    split_pos(idx, hx, ny, i, y, z);
    const int so = (y + z) & 1;
    const T nr = box_nb_sum(u1, i, y, z, nx, ny, nz, so);
    r0[idx] = f0[idx] - ((T)diag.v[box_faces(2 * i + so, y, z, nx, ny, nz)] * u0[idx] - s * nr);
}

template <typename T>
__global__ void __launch_bounds__(kBlock) k_resid_box_vec(const T* __restrict__ u0, const T* __restrict__ u1,
                                                          const T* __restrict__ f0, T* __restrict__ r0, int nx,
                                                          int ny, int nz, T s, BoxCoef diag, const Scalars* sc) {
    if (sc && sc->done) return;
    typedef typename BoxVec<T>::type V;
    constexpr int VW = BoxVec<T>::W;
    const int hx = nx >> 1, hv = hx / VW;
    const unsigned nv = (unsigned)hv * ny * nz;
    const unsigned idx = xcd_block(blockIdx.x, gridDim.x) * blockDim.x + threadIdx.x;
    if (idx >= nv) return;
    int iv, y, z;
    split_pos(idx, hv, ny, iv, y, z);
    const int i0 = iv * VW;
    const int so = (y + z) & 1;
    const V nb = box_nb_vec<T>(u1, i0, y, z, nx, ny, nz, so);
    const size_t row = ((size_t)z * ny + y) * hx;
    const V u = *reinterpret_cast<const V*>(u0 + row + i0);
    const V f = *reinterpret_cast<const V*>(f0 + row + i0);
    const int fyz = (y == 0) + (y + 1 == ny) + (z == 0) + (z + 1 == nz);
    V out;
#pragma unroll
    for (int k = 0; k < VW; ++k)
        out[k] = f[k] - ((T)diag.v[box_faces_vec<VW>(k, i0, hx, so, fyz)] * u[k] - s * nb[k]);
    *reinterpret_cast<V*>(r0 + row + i0) = out;
}

template <typename T>
void launch_resid_red_box(hipStream_t st, const T* u0, const T* u1, const T* f0, T* r0, int nx, int ny, int nz,
                          double s, const BoxCoef& diag, const Scalars* sc) {
    constexpr int VW = BoxVec<T>::W;
    if ((nx / 2) % VW == 0) {
        const unsigned nv = (unsigned)(nx / 2 / VW) * ny * nz;
        hipLaunchKernelGGL(k_resid_box_vec<T>, dim3(nblocks(nv)), dim3(kBlock), 0, st, u0, u1, f0, r0, nx, ny, nz,
                           (T)s, diag, sc);
        return;
    }
    const unsigned nh = (unsigned)(nx / 2) * ny * nz;
    hipLaunchKernelGGL(k_resid_box<T>, dim3(nblocks(nh)), dim3(kBlock), 0, st, u0, u1, f0, r0, nx, ny, nz, (T)s, diag,
                       sc);
}

// Restriction weight of fine cell f = 2X - 1 + b (b = 0..3) for coarse cell X on
// an axis of n fine cells: (1, 3, 3, 1)/8, no fine cell beyond a face, and 2/8
// for a boundary fine cell of a boundary coarse cell (its ghost -u takes 1/8).
template <typename T>
__device__ __forceinline__ T box_rweight(int b, int X, int n) {
    const int f = 2 * X - 1 + b;
    if (f < 0 || f >= n) return (T)0;
    if (b == 0 || b == 3) return (T)0.125;
    if ((b == 1 && f == 0) || (b == 2 && f == n - 1)) return (T)0.25;
    return (T)0.375;
}

// Red fine residual (black cells zero) -> coarse right-hand side: split layout
// with the zero-guess red half-sweep cu0 = cf0 / diag_c(cell), or natural on the
// coarsest level.
template <typename T>
__global__ void __launch_bounds__(kBlock) k_restrict_box(const T* __restrict__ r0, int nx, int ny, int nz,
                                                         T* __restrict__ cf0, T* __restrict__ cf1,
                                                         T* __restrict__ cu0, int coarse_natural, BoxCoef inv_c,
                                                         const Scalars* sc) {
    if (sc && sc->done) return;
    const int cx = nx >> 1, cy = ny >> 1, cz = nz >> 1;
    const unsigned nc = (unsigned)cx * cy * cz;
    const unsigned idx = xcd_block(blockIdx.x, gridDim.x) * blockDim.x + threadIdx.x;
    if (idx >= nc) return;
    const int X = idx % cx;
    const unsigned t = idx / cx;
    const int Y = t % cy, Z = t / cy;
    const int hx = nx >> 1;
    T acc = 0;
#pragma unroll
    for (int c = 0; c < 4; ++c) {
        const T wz = box_rweight<T>(c, Z, nz);
        if (wz == (T)0) continue;
        const int z = 2 * Z - 1 + c;
        T accb = 0;
#pragma unroll
        for (int b = 0; b < 4; ++b) {
            const T wy = box_rweight<T>(b, Y, ny);
            if (wy == (T)0) continue;
            const int y = 2 * Y - 1 + b;
            const T* row = r0 + ((size_t)z * ny + y) * hx;
            const int s0 = (y + z) & 1;  // red cells of this row: x = 2i + s0
            T acca = 0;
#pragma unroll
            for (int a = 0; a < 4; ++a) {
                const int x = 2 * X - 1 + a;
                if ((x & 1) != s0) continue;  // black: zero residual
                const T wx = box_rweight<T>(a, X, nx);
                if (wx != (T)0) acca += wx * row[x >> 1];
            }
            accb += wy * acca;
        }
        acc += wz * accb;
    }
    if (coarse_natural) {
        cf0[idx] = acc;
    } else {
        const size_t j = ((size_t)Z * cy + Y) * (cx >> 1) + (X >> 1);
        if ((X + Y + Z) & 1) {
            cf1[j] = acc;
        } else {
            cf0[j] = acc;
            cu0[j] = acc * (T)inv_c.v[box_faces(X, Y, Z, cx, cy, cz)];
        }
    }
}

// Four consecutive coarse cells X0 .. X0+3 per thread (needs (nx/2) % 4 == 0): per fine
// row one 4-wide load of the red residual plus one edge value. In a row of red parity s0
// the red fine cells of coarse X are 2X-1 (1/8) and 2X+1 (3/8) when s0 = 1, 2X (3/8) and
// 2X+2 (1/8) when s0 = 0; beyond a face the edge value is zero, and the boundary fine cell
// of a boundary coarse cell weighs 2/8.
template <typename T>
__global__ void __launch_bounds__(kBlock) k_restrict_box4(const T* __restrict__ r0, int nx, int ny, int nz,
                                                          T* __restrict__ cf0, T* __restrict__ cf1,
                                                          T* __restrict__ cu0, int coarse_natural, BoxCoef inv_c,
                                                          const Scalars* sc) {
    if (sc && sc->done) return;
    typedef T V4 __attribute__((ext_vector_type(4)));
    typedef T V2 __attribute__((ext_vector_type(2)));
    const int cx = nx >> 1, cy = ny >> 1, cz = nz >> 1, cv = cx >> 2;
    const unsigned n4 = (unsigned)cv * cy * cz;
    const unsigned idx = xcd_block(blockIdx.x, gridDim.x) * blockDim.x + threadIdx.x;
    if (idx >= n4) return;
    const int v = idx % cv;
    const unsigned t = idx / cv;
    const int Y = t % cy, Z = t / cy;
    const int hx = nx >> 1, X0 = 4 * v;
    const T w0 = (T)0.125, w1 = (T)0.375, wb = (T)0.25;
    T acc[4] = {0, 0, 0, 0};
#pragma unroll
    for (int c = 0; c < 4; ++c) {
        const T wz = box_rweight<T>(c, Z, nz);
        if (wz == (T)0) continue;
        const int z = 2 * Z - 1 + c;
        T accb[4] = {0, 0, 0, 0};
#pragma unroll
        for (int b = 0; b < 4; ++b) {
            const T wy = box_rweight<T>(b, Y, ny);
            if (wy == (T)0) continue;
            const int y = 2 * Y - 1 + b;
            const T* row = r0 + ((size_t)z * ny + y) * hx;
            const int s0 = (y + z) & 1;
            const V4 m = *reinterpret_cast<const V4*>(row + X0);
            const T e = s0 ? (X0 > 0 ? row[X0 - 1] : (T)0) : (X0 + 4 < hx ? row[X0 + 4] : (T)0);
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                T val;
                if (s0) {
                    const T wm = (X0 + k == cx - 1) ? wb : w1;  // fine 2X+1 = nx-1 is the boundary cell
                    val = w0 * (k ? m[k - 1] : e) + wm * m[k];
                } else {
                    const T wm = (X0 + k == 0) ? wb : w1;  // fine 2X = 0 is the boundary cell
                    val = wm * m[k] + w0 * (k < 3 ? m[k + 1] : e);
                }
                accb[k] += wy * val;
            }
        }
#pragma unroll
        for (int k = 0; k < 4; ++k) acc[k] += wz * accb[k];
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
        const int fyz = (Y == 0) + (Y + 1 == cy) + (Z == 0) + (Z + 1 == cz);
        const int xa = X0 + pc, xb = X0 + pc + 2;  // the two red coarse cells
        const T ia = (T)inv_c.v[fyz + (xa == 0) + (xa == cx - 1)];
        const T ib = (T)inv_c.v[fyz + (xb == 0) + (xb == cx - 1)];
        *reinterpret_cast<V2*>(cu0 + j) = V2{red[0] * ia, red[1] * ib};
    }
}

template <typename T>
void launch_restrict_box(hipStream_t st, const T* r0, int nx, int ny, int nz, T* cf0, T* cf1, T* cu0,
                         int coarse_natural, const BoxCoef& inv_c, const Scalars* sc) {
    if ((nx / 2) % 4 == 0) {
        const unsigned n4 = (unsigned)(nx / 8) * (ny / 2) * (nz / 2);
        hipLaunchKernelGGL(k_restrict_box4<T>, dim3(nblocks(n4)), dim3(kBlock), 0, st, r0, nx, ny, nz, cf0, cf1, cu0,
                           coarse_natural, inv_c, sc);
        return;
    }
    const unsigned nc = (unsigned)(nx / 2) * (ny / 2) * (nz / 2);
    hipLaunchKernelGGL(k_restrict_box<T>, dim3(nblocks(nc)), dim3(kBlock), 0, st, r0, nx, ny, nz, cf0, cf1, cu0,
                       coarse_natural, inv_c, sc);
}

namespace {

template <typename T>
__device__ __forceinline__ T box_coarse_at(const T* __restrict__ c0, const T* __restrict__ c1, int nat, int X, int Y,
                                           int Z, int cx, int cy) {
    if (nat) return c0[((size_t)Z * cy + Y) * cx + X];
    const size_t j = ((size_t)Z * cy + Y) * (cx >> 1) + (X >> 1);
    return ((X + Y + Z) & 1) ? c1[j] : c0[j];
}

// Interpolation weights of fine cell f on an axis of nc coarse cells: 3/4 of its
// parent f/2 and 1/4 of the next coarse cell towards f; beyond a face that cell
// is the ghost -u of the parent, so the parent takes 1/2 (the second index is
// then the parent itself with weight 0, which keeps the read in bounds).
template <typename T>
__device__ __forceinline__ void box_pweights(int f, int nc, int& I0, int& I1, T& w0, T& w1) {
    I0 = f >> 1;
    I1 = (f & 1) ? I0 + 1 : I0 - 1;
    if (I1 < 0 || I1 >= nc) {
        I1 = I0;
        w0 = (T)0.5;
        w1 = (T)0;
    } else {
        w0 = (T)0.75;
        w1 = (T)0.25;
    }
}

}  // namespace

// Red-only trilinear correction (the post-smoothing's first black half-sweep
// overwrites every black value without reading it).
template <typename T>
__global__ void __launch_bounds__(kBlock) k_prolong_red_box(const T* __restrict__ cu0, const T* __restrict__ cu1,
                                                            int nat, T* __restrict__ u0, int nx, int ny, int nz,
                                                            const Scalars* sc) {
    if (sc && sc->done) return;
    const int hx = nx >> 1;
    const unsigned nh = (unsigned)hx * ny * nz;
    const unsigned idx = xcd_block(blockIdx.x, gridDim.x) * blockDim.x + threadIdx.x;
    if (idx >= nh) return;
    int i, y, z;
    split_pos(idx, hx, ny, i, y, z);
    const int cx = nx >> 1, cy = ny >> 1, cz = nz >> 1;
    int I0, I1, J0, J1, K0, K1;
    T a0, a1, b0, b1, c0, c1;
    box_pweights<T>(2 * i + ((y + z) & 1), cx, I0, I1, a0, a1);
    box_pweights<T>(y, cy, J0, J1, b0, b1);
    box_pweights<T>(z, cz, K0, K1, c0, c1);
    auto row = [&](int J, int K) {
        return a0 * box_coarse_at(cu0, cu1, nat, I0, J, K, cx, cy) + a1 * box_coarse_at(cu0, cu1, nat, I1, J, K, cx, cy);
    };
    const T v00 = row(J0, K0), v10 = row(J1, K0), v01 = row(J0, K1), v11 = row(J1, K1);
    u0[idx] += c0 * (b0 * v00 + b1 * v10) + c1 * (b0 * v01 + b1 * v11);
}

// The coarse values c(i0 + d), d = 0 .. VW-1, of row (Y, Z) of a coarse box level, and
// the next one on the fine cells' side, e = c(i0 + VW) (s = 1) or c(i0 - 1) (s = 0); past
// a face e is the end cell's own value (its weight is then 0). In the split layout i0 is
// even, so c(i0 + d) is element i0/2 + d/2 of c1 when d + Y + Z is odd and of c0
// otherwise: one VW/2-wide load from each half gives the run.
template <typename T>
__device__ __forceinline__ void box_coarse_row(const T* __restrict__ c0, const T* __restrict__ c1, int nat, int Y,
                                               int Z, int i0, int s, int cx, int cy, T (&m)[BoxVec<T>::W], T& e) {
    constexpr int VW = BoxVec<T>::W, HW = VW / 2;
    struct alignas(sizeof(T) * HW) Half { T v[HW]; };
    if (nat) {
        const T* r = c0 + ((size_t)Z * cy + Y) * cx;
#pragma unroll
        for (int d = 0; d < VW; ++d) m[d] = r[i0 + d];
    } else {
        const size_t rb = ((size_t)Z * cy + Y) * (cx >> 1);
        const int p = (Y + Z) & 1;
        const Half a = *reinterpret_cast<const Half*>(c0 + rb + (i0 >> 1));
        const Half b = *reinterpret_cast<const Half*>(c1 + rb + (i0 >> 1));
#pragma unroll
        for (int d = 0; d < VW; ++d) m[d] = ((d + p) & 1) ? b.v[d >> 1] : a.v[d >> 1];
    }
    // clamped: past a face the end cell itself
    const int X = s ? min(i0 + VW, cx - 1) : max(i0 - 1, 0);
    e = box_coarse_at(c0, c1, nat, X, Y, Z, cx, cy);
}

// Vector form: VW red cells of a split row per thread, one 16-byte read-modify-write of
// u0; the cells share their coarse rows, each read once (VW + 1 values).
template <typename T>
__global__ void __launch_bounds__(kBlock) k_prolong_red_box_vec(const T* __restrict__ cu0, const T* __restrict__ cu1,
                                                                int nat, T* __restrict__ u0, int nx, int ny, int nz,
                                                                const Scalars* sc) {
    if (sc && sc->done) return;
    typedef typename BoxVec<T>::type V;
    constexpr int VW = BoxVec<T>::W;
    const int hx = nx >> 1, hv = hx / VW;
    const unsigned nv = (unsigned)hv * ny * nz;
    const unsigned idx = xcd_block(blockIdx.x, gridDim.x) * blockDim.x + threadIdx.x;
    if (idx >= nv) return;
    int iv, y, z;
    split_pos(idx, hv, ny, iv, y, z);
    const int i0 = iv * VW;
    const int cx = nx >> 1, cy = ny >> 1, cz = nz >> 1;
    const int s0 = (y + z) & 1;  // red cell x = 2i + s0: coarse parent i
    int J0, J1, K0, K1;
    T b0, b1, c0, c1;
    box_pweights<T>(y, cy, J0, J1, b0, b1);
    box_pweights<T>(z, cz, K0, K1, c0, c1);
    T m00[VW], m10[VW], m01[VW], m11[VW], e00, e10, e01, e11;
    box_coarse_row<T>(cu0, cu1, nat, J0, K0, i0, s0, cx, cy, m00, e00);
    box_coarse_row<T>(cu0, cu1, nat, J1, K0, i0, s0, cx, cy, m10, e10);
    box_coarse_row<T>(cu0, cu1, nat, J0, K1, i0, s0, cx, cy, m01, e01);
    box_coarse_row<T>(cu0, cu1, nat, J1, K1, i0, s0, cx, cy, m11, e11);
    const size_t row = ((size_t)z * ny + y) * hx;
    V u = *reinterpret_cast<const V*>(u0 + row + i0);
#pragma unroll
    for (int k = 0; k < VW; ++k) {
        int I0, I1;
        T a0, a1;
        box_pweights<T>(2 * (i0 + k) + s0, cx, I0, I1, a0, a1);
        // the value at I1: the side neighbour, or past a face the cell itself (weight 0)
        const T n00 = s0 ? (k + 1 < VW ? m00[k + 1] : e00) : (k > 0 ? m00[k - 1] : e00);
        const T n10 = s0 ? (k + 1 < VW ? m10[k + 1] : e10) : (k > 0 ? m10[k - 1] : e10);
        const T n01 = s0 ? (k + 1 < VW ? m01[k + 1] : e01) : (k > 0 ? m01[k - 1] : e01);
        const T n11 = s0 ? (k + 1 < VW ? m11[k + 1] : e11) : (k > 0 ? m11[k - 1] : e11);
        const T v00 = a0 * m00[k] + a1 * n00, v10 = a0 * m10[k] + a1 * n10;
        const T v01 = a0 * m01[k] + a1 * n01, v11 = a0 * m11[k] + a1 * n11;
        u[k] += c0 * (b0 * v00 + b1 * v10) + c1 * (b0 * v01 + b1 * v11);
    }
    *reinterpret_cast<V*>(u0 + row + i0) = u;
}

template <typename T>
void launch_prolong_red_box(hipStream_t st, const T* cu0, const T* cu1, int coarse_natural, T* u0, int nx, int ny,
                            int nz, const Scalars* sc) {
    constexpr int VW = BoxVec<T>::W;
    if ((nx / 2) % VW == 0) {
        const unsigned nv = (unsigned)(nx / 2 / VW) * ny * nz;
        hipLaunchKernelGGL(k_prolong_red_box_vec<T>, dim3(nblocks(nv)), dim3(kBlock), 0, st, cu0, cu1, coarse_natural,
                           u0, nx, ny, nz, sc);
        return;
    }
    const unsigned nh = (unsigned)(nx / 2) * ny * nz;
    hipLaunchKernelGGL(k_prolong_red_box<T>, dim3(nblocks(nh)), dim3(kBlock), 0, st, cu0, cu1, coarse_natural, u0, nx,
                       ny, nz, sc);
}

// ---------------------------------------------------------------------------
// Coarse tail of the box V-cycle: every level from t down in LDS of one work-group
// (natural layout), the steps of the per-level box kernels in their order: zero
// guess, R B R B pre-smoothing, red residual, restriction, the coarsest dense
// solve, correction, B R B R post-smoothing. The per-cell diagonal is
// alpha + s (6 + faces) = d.diag[l] + faces * s.
namespace {

// j -> (a, b, c) for row-major dims (na, nb, *); shifts and masks when both are powers of two
struct TailPos {
    int na, nb, la, lab;
    bool p2;
    __device__ __forceinline__ TailPos(int a, int b) : na(a), nb(b) {
        p2 = ((a & (a - 1)) == 0) && ((b & (b - 1)) == 0);
        la = __ffs(a) - 1;
        lab = la + __ffs(b) - 1;
    }
    __device__ __forceinline__ void operator()(int j, int& a, int& b, int& c) const {
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
};

template <typename T>
__device__ __forceinline__ T tail_nb_box(const T* u, int x, int y, int z, int nx, int ny, int nz) {
    const int row = (z * ny + y) * nx + x;
    const int plane = nx * ny;
    const T xm = x > 0 ? u[row - 1] : (T)0;
    const T xp = x + 1 < nx ? u[row + 1] : (T)0;
    const T ym = y > 0 ? u[row - nx] : (T)0;
    const T yp = y + 1 < ny ? u[row + nx] : (T)0;
    const T zm = z > 0 ? u[row - plane] : (T)0;
    const T zp = z + 1 < nz ? u[row + plane] : (T)0;
    return ((xm + xp) + (ym + yp)) + (zm + zp);
}

// inverse diagonals of a level for 0..3 faces, selected without a runtime-indexed array
template <typename T>
struct TailInv {
    T i0, i1, i2, i3;
    __device__ __forceinline__ TailInv(T dg0, T s)
        : i0((T)1 / dg0), i1((T)1 / (dg0 + s)), i2((T)1 / (dg0 + 2 * s)), i3((T)1 / (dg0 + 3 * s)) {}
    __device__ __forceinline__ T operator()(int f) const { return f == 0 ? i0 : (f == 1 ? i1 : (f == 2 ? i2 : i3)); }
};

template <typename T>
__device__ __forceinline__ void tail_gs_box(T* u, const T* f, int nx, int ny, int nz, int color, T s,
                                            const TailInv<T>& inv) {
    const int hx = nx >> 1, nh = hx * ny * nz;
    const TailPos dec(hx, ny);
    for (int j = threadIdx.x; j < nh; j += blockDim.x) {
        int i, y, z;
        dec(j, i, y, z);
        const int x = 2 * i + ((y + z + color) & 1);
        const int k = (z * ny + y) * nx + x;
        u[k] = (f[k] + s * tail_nb_box(u, x, y, z, nx, ny, nz)) * inv(box_faces(x, y, z, nx, ny, nz));
    }
    __syncthreads();
}

}  // namespace

template <typename T>
__global__ void __launch_bounds__(kFinBlock) k_tail_box(const T* __restrict__ f0g, const T* __restrict__ f1g,
                                                        T* __restrict__ u0g, T* __restrict__ u1g, TailDesc d,
                                                        const double* __restrict__ cinv, const Scalars* sc) {
    if (sc && sc->done) return;
    extern __shared__ __align__(16) unsigned char smem[];
    auto U_ = [&](int l) { return reinterpret_cast<T*>(smem + d.off_u[l]); };
    auto F_ = [&](int l) { return reinterpret_cast<T*>(smem + d.off_f[l]); };
    auto R_ = [&](int l) { return reinterpret_cast<T*>(smem + d.off_r[l]); };
    const int L = d.nlev - 1;  // coarsest, natural, m cells
    {
        // split (red, black) global arrays of the first tail level -> natural LDS
        const int nx = d.nx[0], ny = d.ny[0], hx = nx >> 1, nh = hx * ny * d.nz[0];
        T* F0 = F_(0);
        const TailPos dec(hx, ny);
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
        T* U = U_(l);
        T* F = F_(l);
        T* R = R_(l);
        const T s = (T)d.s[l], dg0 = (T)d.diag[l];
        const TailInv<T> inv(dg0, s);
        for (int j = threadIdx.x; j < n; j += blockDim.x) U[j] = (T)0;
        __syncthreads();
        tail_gs_box(U, F, nx, ny, nz, 0, s, inv);
        tail_gs_box(U, F, nx, ny, nz, 1, s, inv);
        tail_gs_box(U, F, nx, ny, nz, 0, s, inv);
        tail_gs_box(U, F, nx, ny, nz, 1, s, inv);
        const TailPos dec(nx, ny);
        for (int j = threadIdx.x; j < n; j += blockDim.x) {
            int x, y, z;
            dec(j, x, y, z);
            const T dg = dg0 + (T)box_faces(x, y, z, nx, ny, nz) * s;
            R[j] = ((x + y + z) & 1) ? (T)0 : F[j] - (dg * U[j] - s * tail_nb_box(U, x, y, z, nx, ny, nz));
        }
        __syncthreads();
        const int cx = nx >> 1, cy = ny >> 1, nc = cx * cy * (nz >> 1);
        T* Fc = F_(l + 1);
        const TailPos cdec(cx, cy);
        for (int j = threadIdx.x; j < nc; j += blockDim.x) {
            int X, Y, Z;
            cdec(j, X, Y, Z);
            T acc = 0;
#pragma unroll
            for (int c = 0; c < 4; ++c) {
                const T wz = box_rweight<T>(c, Z, nz);
                if (wz == (T)0) continue;
                T accb = 0;
#pragma unroll
                for (int b = 0; b < 4; ++b) {
                    const T wy = box_rweight<T>(b, Y, ny);
                    if (wy == (T)0) continue;
                    const T* rr = R + ((2 * Z - 1 + c) * ny + (2 * Y - 1 + b)) * nx;
                    T acca = 0;
#pragma unroll
                    for (int a = 0; a < 4; ++a) {
                        const T wx = box_rweight<T>(a, X, nx);
                        if (wx != (T)0) acca += wx * rr[2 * X - 1 + a];
                    }
                    accb += wy * acca;
                }
                acc += wz * accb;
            }
            Fc[j] = acc;
        }
        __syncthreads();
    }
    {
        // one wave per row of the dense inverse
        const T* Fl = F_(L);
        T* Ul = U_(L);
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
        const T* C = U_(l + 1);
        T* U = U_(l);
        const T* F = F_(l);
        const TailPos dec(nx, ny);
        for (int j = threadIdx.x; j < n; j += blockDim.x) {
            int x, y, z;
            dec(j, x, y, z);
            int I0, I1, J0, J1, K0, K1;
            T a0, a1, b0, b1, c0, c1;
            box_pweights<T>(x, cx, I0, I1, a0, a1);
            box_pweights<T>(y, cy, J0, J1, b0, b1);
            box_pweights<T>(z, cz, K0, K1, c0, c1);
            auto line = [&](int J, int K) {
                const T* cr = C + (K * cy + J) * cx;
                return a0 * cr[I0] + a1 * cr[I1];
            };
            U[j] += c0 * (b0 * line(J0, K0) + b1 * line(J1, K0)) + c1 * (b0 * line(J0, K1) + b1 * line(J1, K1));
        }
        __syncthreads();
        const T s = (T)d.s[l];
        const TailInv<T> inv((T)d.diag[l], s);
        tail_gs_box(U, F, nx, ny, nz, 1, s, inv);
        tail_gs_box(U, F, nx, ny, nz, 0, s, inv);
        tail_gs_box(U, F, nx, ny, nz, 1, s, inv);
        tail_gs_box(U, F, nx, ny, nz, 0, s, inv);
    }
    {
        const int nx = d.nx[0], ny = d.ny[0], hx = nx >> 1, nh = hx * ny * d.nz[0];
        const T* U0 = U_(0);
        const TailPos dec(hx, ny);
        for (int j = threadIdx.x; j < nh; j += blockDim.x) {
            int i, y, z;
            dec(j, i, y, z);
            const int row = (z * ny + y) * nx, par = (y + z) & 1;
            u0g[j] = U0[row + 2 * i + par];
            u1g[j] = U0[row + 2 * i + (par ^ 1)];
        }
    }
}

template <typename T>
void launch_tail_box(hipStream_t st, const T* f0, const T* f1, T* u0, T* u1, const TailDesc& d, const double* cinv,
                     const Scalars* sc) {
    hipLaunchKernelGGL(k_tail_box<T>, dim3(1), dim3(kFinBlock), d.lds_bytes, st, f0, f1, u0, u1, d, cinv, sc);
}

template <typename T>
hipError_t tail_box_set_lds(size_t bytes) {
    return hipFuncSetAttribute((const void*)k_tail_box<T>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
}

#define BRD_BOX_INST(T)                                                                                              \
    template void launch_enter_box<T>(hipStream_t, const double*, T*, T*, T*, int, int, int, const BoxCoef&,         \
                                      const Scalars*);                                                               \
    template void launch_gs_box<T>(hipStream_t, T*, const T*, const T*, int, int, int, int, double, const BoxCoef&,  \
                                   const Scalars*);                                                                  \
    template void launch_resid_red_box<T>(hipStream_t, const T*, const T*, const T*, T*, int, int, int, double,      \
                                          const BoxCoef&, const Scalars*);                                           \
    template void launch_restrict_box<T>(hipStream_t, const T*, int, int, int, T*, T*, T*, int, const BoxCoef&,      \
                                         const Scalars*);                                                            \
    template void launch_prolong_red_box<T>(hipStream_t, const T*, const T*, int, T*, int, int, int, const Scalars*); \
    template void launch_tail_box<T>(hipStream_t, const T*, const T*, T*, T*, const TailDesc&, const double*,       \
                                     const Scalars*);                                                                \
    template hipError_t tail_box_set_lds<T>(size_t);
BRD_BOX_INST(float)
BRD_BOX_INST(double)
#undef BRD_BOX_INST

}  // namespace brd
