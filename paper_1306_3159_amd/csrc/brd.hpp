// Internal declarations of the blob_rd HIP library (gfx950).
//
// Data layout in device memory:
//  * FP64 grid vectors (Krylov iterates, residuals, right-hand sides) are in
//    natural order [z][y][x], x fastest, as the public ABI exposes them.
//  * Multigrid levels are stored red/black split: level l with dims
//    (nx, ny, nz), nx even, keeps two arrays per field, one per colour
//    (colour = (x + y + z) mod 2, red = 0), each [z][y][nx/2]. Cell (x, y, z)
//    of colour c sits at index x/2 of row (y, z) of array c. A Gauss-Seidel
//    half-sweep then reads the other colour's array and writes its own with
//    unit stride. The coarsest level (<= 512 cells, possibly odd) is natural.
//  * Blob data are structure-of-arrays in original blob order plus a
//    permutation that sorts blobs by the grid tile of their base cell.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

namespace brd {

constexpr int kBlock = 256;
constexpr int kMaxTuneBlock = 512;  // largest work-group the autotuner may pick
constexpr int kFinBlock = 1024;
constexpr int kMaxLevels = 16;
constexpr int kMaxCoarse = 512;
constexpr int kMaxCoarseCols = 256;  // columns of the Schur preconditioner's Fourier coarse level
constexpr int kCoarseChunk = 2048;   // rows per work-group in the coarse level's dot products
constexpr int kStageBlobs = 128;   // candidate blobs staged in LDS per pass of the spread planner

// Device-resident scalars of one CG solve. Every kernel of an iteration reads
// `done` first and returns if it is set, so the host can enqueue iterations
// without waiting for convergence.
struct Scalars {
    double rz;        // z . r of the current iterate (with the constant shift)
    double pq;        // p . B p
    double alpha;     // CG step
    double beta;      // CG direction update (Polak-Ribiere form)
    double rr;        // r . r
    double rsum;      // sum r
    double qsum;      // sum q
    double tol2;      // stop when rr <= tol2
    double shift;     // constant added to the V-cycle output z (null-space handling)
    double mean_r;    // mean removed from r before the V-cycle (projected problems)
    double mean_next; // mean of the next r predicted from sum r and sum q (fused update + V-cycle entry)
    double inv_ncell; // 1 / (nx ny nz)
    double eBe_inv;   // 1 / (e^T B e) for the reactive alpha = 0 constant mode (0 otherwise)
    double rr0;       // r . r of the initial residual
    double gg;        // right-hand side g . g
    int32_t done;     // 1: converged (or failed); kernels become no-ops
    int32_t iters;    // completed CG iterations
    int32_t project;  // 1: alpha = 0 problem, work on mean-zero vectors
    int32_t status;   // 0 ok, 1 breakdown/non-finite
    int32_t xzero;    // 1: x starts at zero and the first update writes it (no prior fill)
};

// Device-resident scalars of the Schur GMRES (single work-group kernels).
struct GmresScalars {
    double beta;      // initial residual norm of the current cycle
    double res;       // current residual estimate |g_{k+1}|
    double hk1;       // last subdiagonal entry
    int32_t k;        // columns in the current cycle
    int32_t status;
};

// Longest restart of the flexible GMRES on the block saddle system.
constexpr int kFgMaxRestart = 1024;

// Levels handled by the single-work-group coarse tail (index 0 = first tail
// level, last = coarsest). LDS byte offsets of u, f, r per level.
struct TailDesc {
    int nlev;
    int m;
    int nx[kMaxLevels], ny[kMaxLevels], nz[kMaxLevels];
    double s[kMaxLevels], diag[kMaxLevels], inv_diag[kMaxLevels];
    unsigned off_u[kMaxLevels], off_f[kMaxLevels], off_r[kMaxLevels];
    unsigned lds_bytes;
};

// Learned preconditioner network: flat float32 parameter vector
// [W1 (64 x 12, row = output) | b1 | W2 (64 x 64) | b2 | w3 | b3].
constexpr int kNetFeat = 12;
constexpr int kOffW1 = 0, kOffB1 = 768, kOffW2 = 832, kOffB2 = 4928, kOffW3 = 4992, kOffB3 = 5056;
constexpr int kNetParams = 5057;
constexpr float kNuScale = 0.25f;  // neighbour counts enter the network as nu / 4

struct NetDev {
    const float* P;     // float32 masters
    const __bf16* W1b;  // [64][16] bfloat16, columns >= 10 zero
    const __bf16* W2b;  // [64][64] bfloat16
    const __bf16* w3b;  // [64] bfloat16
};

struct PairGeom {
    double box[3];  // box edge per axis (x, y, z)
    double h;
    double rc;      // pair cutoff
    int ncx, ncy, ncz;  // pair-search cells per axis
    const float* nu;    // per blob: other blobs within rc / 2 (network input; null while the list is built)
};

struct BlobGeom {
    int nx, ny, nz;
    int tx, ty, tz;      // tile edge per axis (divides the grid edge)
    int ntx, nty, ntz;   // tiles per axis
    double h;
    int w;
};

// Contribution lists of the spread: n touched cells, cell[k] its grid index,
// entries ptr[k] .. ptr[k+1] of (blob[e], weight w[e]).
struct SpreadLists {
    int n;
    const int* cell;
    const int* ptr;
    const int* blob;
    const double* w;
};
// Multipliers a spread takes: lam[b] + c2 lam2[b] + shift (lam, lam2 may be null).
struct SpreadMult {
    const double* lam;
    const double* lam2;
    double c2;
    double shift;
};

// A box held at a fixed face value (Dirichlet): the homogeneous operator takes the
// ghost beyond a face as minus the boundary cell, so a cell touching f faces has
// the diagonal alpha + s (6 + f) and no neighbour term across them. v[f] holds
// the per-cell coefficient (diagonal or its inverse) for f = 0..3.
struct BoxCoef {
    double v[4];
};

// Logical block of a launch: partial-sum slot b of nb. Solo kernels pass
// (blockIdx.x, gridDim.x); batched kernels pass an instance's local slot, so
// every instance's partition of work and of partial sums is the solo one.
struct Blk {
    unsigned b, nb;
};

// One instance's slice of a batched launch: global blocks [block0, block0 + nb)
// (block0 a multiple of 8, so a slot keeps the XCD of its solo launch).
struct BatchEntry {
    unsigned block0, nb;
    int inst;
    int pad;
};

// Everything a batched CG iteration reads about one instance (device memory).
struct InstDev {
    Scalars* sc;
    double* part;
    double *x, *r, *p, *q;               // CG vectors of the current solve
    double alpha;                         // operator alpha I - D L (+ S kappa J)
    int nx, ny, nz, nlev, t;              // level 0 dims, levels, first tail level
    int np_apply, np_update, np_dots;     // partial slots of the three reductions
    void* lv[kMaxLevels][5];              // split level arrays u0, u1, f0, f1, r0
    int lnx[kMaxLevels], lny[kMaxLevels], lnz[kMaxLevels];
    double ls[kMaxLevels], ldiag[kMaxLevels];  // D / h_l^2 and alpha + 6 s_l
    int blobs, N;                         // blob term in the operator (reactive)
    BlobGeom geom;
    const int* base;
    const double* wts;
    const int* offsets;
    const int* perm;
    const double* kappa;
    double* jx;
    double* mu;
    double inv_h3;
    int ntouched;                         // spread contribution lists (touched cells, entries)
    const int* tcell;
    const int* tptr;
    const int* tblob;
    const double* tw;
    const double* cinv;                   // coarsest (pseudo-)inverse for alpha
    TailDesc tail;
};

struct LevelDims {
    int nx, ny, nz;   // cells
    int hx;           // nx / 2 (split levels)
    double h;         // spacing at this level
};

// ---- helpers -------------------------------------------------------------
__device__ __forceinline__ int wrapi(int i, int n) { return i < 0 ? i + n : (i >= n ? i - n : i); }

// number of box faces cell (x, y, z) touches (at most one per axis for edges >= 2)
__device__ __forceinline__ int box_faces(int x, int y, int z, int nx, int ny, int nz) {
    return (x == 0) + (x == nx - 1) + (y == 0) + (y == ny - 1) + (z == 0) + (z == nz - 1);
}

// Value of cell (X, Y, Z) of a red/black split level (colour (X + Y + Z) mod 2,
// index X/2 of row (Y, Z) of its colour array, hx = nx/2) as a double.
template <typename T>
__device__ __forceinline__ double split_at(const T* __restrict__ z0, const T* __restrict__ z1, int X, int Y, int Z,
                                           int hx, int ny) {
    const size_t j = ((size_t)Z * ny + Y) * hx + (X >> 1);
    return ((X + Y + Z) & 1) ? (double)z1[j] : (double)z0[j];
}

// g - (alpha c - D L c) at natural cell (X, Y, Z) of the periodic level 0 (nx even, s = D / h^2)
// with c in the split layout, in FP64 on c's values: the stencil association of the natural
// two-cell form (x pair, y pair, z pair, then the centre).
template <typename T>
__device__ __forceinline__ double split_resid(const double* __restrict__ g, const T* __restrict__ c0,
                                              const T* __restrict__ c1, int X, int Y, int Z, int nx, int ny, int nz,
                                              double alpha, double s) {
    const int hx = nx >> 1;
    const double c = split_at(c0, c1, X, Y, Z, hx, ny);
    const double xl = split_at(c0, c1, wrapi(X - 1, nx), Y, Z, hx, ny);
    const double xr = split_at(c0, c1, wrapi(X + 1, nx), Y, Z, hx, ny);
    const double ym = split_at(c0, c1, X, wrapi(Y - 1, ny), Z, hx, ny);
    const double yp = split_at(c0, c1, X, wrapi(Y + 1, ny), Z, hx, ny);
    const double zm = split_at(c0, c1, X, Y, wrapi(Z - 1, nz), hx, ny);
    const double zp = split_at(c0, c1, X, Y, wrapi(Z + 1, nz), hx, ny);
    const double a = alpha * c - s * ((xl + xr) + (ym + yp) + (zm + zp) - 6.0 * c);
    return g[((size_t)Z * ny + Y) * nx + X] - a;
}

// Blocks are dispatched to the 8 XCDs round-robin; this remaps the hardware
// block id so each XCD works on one contiguous eighth of the index space,
// keeping neighbouring rows and planes in the same XCD's L2.
__device__ __forceinline__ unsigned xcd_block(unsigned b, unsigned nb) {
    unsigned full = nb >> 3, rem = nb & 7u, xcd = b & 7u, local = b >> 3;
    return xcd * full + (xcd < rem ? xcd : rem) + local;
}

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

// Deterministic block reduction of K values; thread k < K writes block
// partial k to part[k * nparts + slot].
template <int K>
__device__ __forceinline__ void block_partials(double (&v)[K], double* part, unsigned nparts, unsigned slot) {
    __shared__ double sh[K][16];
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6, nw = (blockDim.x + 63) >> 6;
#pragma unroll
    for (int k = 0; k < K; ++k) v[k] = wave_sum(v[k]);
    if (lane == 0)
#pragma unroll
        for (int k = 0; k < K; ++k) sh[k][wid] = v[k];
    __syncthreads();
    if (threadIdx.x < K) {
        double s = 0.0;
        for (int w = 0; w < nw; ++w) s += sh[threadIdx.x][w];
        part[(size_t)threadIdx.x * nparts + slot] = s;
    }
}

// Sum over one work-group (wave sums, then the waves in order); every thread
// gets the total.
__device__ __forceinline__ double wg_sum(double s) {
    __shared__ double sh[kFinBlock / 64];
    s = wave_sum(s);
    __syncthreads();
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = s;
    __syncthreads();
    double t = 0.0;
    for (int w = 0; w < (int)(blockDim.x >> 6); ++w) t += sh[w];
    __syncthreads();
    return t;
}

inline unsigned nblocks(size_t n, int bs = kBlock) { return (unsigned)((n + bs - 1) / bs); }

// Reductions over grid vectors use at most kRedBlocks blocks, each owning one
// contiguous chunk of the index space, so the finalize reads few partials.
constexpr unsigned kRedBlocks = 4096;
inline unsigned red_blocks(size_t n) {
    const unsigned nb = nblocks(n);
    return nb < kRedBlocks ? nb : kRedBlocks;
}
// Entry of a batched launch that owns global block g (entries sorted by block0).
__device__ __forceinline__ int batch_entry(const BatchEntry* e, int n, unsigned g) {
    int lo = 0, hi = n - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (e[mid].block0 <= g) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

// A batched launch's work list, rebuilt for the instances taking part in each
// round: `total` virtual blocks over `n` entries (the BatchEntry array follows
// the header). Launches have a fixed grid that strides over the virtual blocks.
struct BatchTab {
    unsigned total;
    int n;
    int pad0, pad1;
};
__device__ __forceinline__ const BatchEntry* tab_entries(const BatchTab* t) {
    return reinterpret_cast<const BatchEntry*>(t + 1);
}

// The instance and local block of virtual block g, or null when g is padding,
// the instance is not gated in, or its solve is done (uniform per block, so
// callers may skip barriers together).
__device__ __forceinline__ const InstDev* batch_slot(const InstDev* inst, const int* gate, const BatchEntry* ent,
                                                     int nent, unsigned g, Blk& blk) {
    const BatchEntry e = ent[batch_entry(ent, nent, g)];
    const unsigned b = g - e.block0;
    if (b >= e.nb || !gate[e.inst]) return nullptr;
    const InstDev* I = inst + e.inst;
    if (I->sc->done) return nullptr;
    blk.b = b;
    blk.nb = e.nb;
    return I;
}

// chunk [lo, hi) of logical block b of nb over n items (chunks are multiples of blockDim)
__device__ __forceinline__ void chunk_of(unsigned b, unsigned nb, unsigned n, unsigned* lo, unsigned* hi) {
    const unsigned per = ((n + nb - 1) / nb + blockDim.x - 1) / blockDim.x * blockDim.x;
    const unsigned l = b * per;
    *lo = l < n ? l : n;
    *hi = l + per < n ? l + per : n;
}

}  // namespace brd
