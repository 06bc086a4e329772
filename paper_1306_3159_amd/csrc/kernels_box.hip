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

template <typename T>
void launch_gs_box(hipStream_t st, T* uc, const T* uo, const T* fc, int nx, int ny, int nz, int color, double s,
                   const BoxCoef& inv, const Scalars* sc) {
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
void launch_resid_red_box(hipStream_t st, const T* u0, const T* u1, const T* f0, T* r0, int nx, int ny, int nz,
                          double s, const BoxCoef& diag, const Scalars* sc) {
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

template <typename T>
void launch_restrict_box(hipStream_t st, const T* r0, int nx, int ny, int nz, T* cf0, T* cf1, T* cu0,
                         int coarse_natural, const BoxCoef& inv_c, const Scalars* sc) {
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

template <typename T>
void launch_prolong_red_box(hipStream_t st, const T* cu0, const T* cu1, int coarse_natural, T* u0, int nx, int ny,
                            int nz, const Scalars* sc) {
    const unsigned nh = (unsigned)(nx / 2) * ny * nz;
    hipLaunchKernelGGL(k_prolong_red_box<T>, dim3(nblocks(nh)), dim3(kBlock), 0, st, cu0, cu1, coarse_natural, u0, nx,
                       ny, nz, sc);
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
    template void launch_prolong_red_box<T>(hipStream_t, const T*, const T*, int, T*, int, int, int, const Scalars*);
BRD_BOX_INST(float)
BRD_BOX_INST(double)
#undef BRD_BOX_INST

}  // namespace brd
