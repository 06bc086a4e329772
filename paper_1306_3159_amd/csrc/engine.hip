// Host engine and C-ABI of blob_rd.
//
// Solvers (arXiv:1306.3159):
//  * reactive system (alpha I - D L + S kappa J) c = f (eqs. unsteady_system,
//    steady_state) by CG preconditioned with one multigrid V-cycle for
//    alpha I - D L (Sec. III.E, eq. Pinv_Poisson). CG scalars stay on the
//    device; the direction update uses the Polak-Ribiere form so an FP32
//    V-cycle (slightly nonlinear in rounding) is tolerated. For alpha = 0 the
//    preconditioner is P MG(P r) + e (e^T r)/(e^T B e), P = I - e e^T/n;
//  * absorbing saddle point (eq. saddle_point, zeta = 1, xi = 1/dV_f) by
//    Schur-complement GMRES(m) with modified Gram-Schmidt on
//    G = J (alpha I - D L)^+ S (eqs. c_exact, r_schur); for alpha = 0 the
//    periodic null space is handled as in Appendix A: the mean sink strength
//    is fixed by the total source, GMRES works on mean-zero N-vectors and
//    the mean concentration follows from J c = 0;
//  * backward-Euler steps (eq. c_np1).
// Every solve ends with an FP64 residual of the returned answer and, when
// that misses the target, iterative refinement on the residual equations.
#include <hip/hip_runtime.h>
#include <unistd.h>

#include <algorithm>
#include <atomic>
#include <thread>
#include <mutex>
#include <condition_variable>
#include <chrono>
#include <type_traits>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <stdexcept>
#include <string>
#include <vector>

#include "../../include/blob_rd.h"
#include "launch.hpp"

using namespace brd;

namespace {

thread_local std::string g_last_error = "";

struct Err : std::runtime_error {
    int code;
    Err(int c, const std::string& m) : std::runtime_error(m), code(c) {}
};

#define HIPCHK(x)                                                                                      \
    do {                                                                                               \
        hipError_t e_ = (x);                                                                           \
        if (e_ != hipSuccess)                                                                          \
            throw Err(BLOB_RD_EDEVICE, std::string(#x ": ") + hipGetErrorString(e_));                  \
    } while (0)

size_t align_up(size_t v) { return (v + 255) & ~(size_t)255; }

int level_dims(int nx, int ny, int nz, LevelDims* out) {
    int l = 0;
    for (;;) {
        if (l >= kMaxLevels) return -1;
        out[l].nx = nx;
        out[l].ny = ny;
        out[l].nz = nz;
        out[l].hx = nx / 2;
        ++l;
        if ((nx & 1) || (ny & 1) || (nz & 1) || nx <= 4 || ny <= 4 || nz <= 4) break;
        nx /= 2;
        ny /= 2;
        nz /= 2;
    }
    return l;
}

int tile_edge(int n) {
    if (n % 8 == 0) return 8;
    for (int d = 7; d >= 3; --d)
        if (n % d == 0) return d;
    return -1;
}

// Workspace plan: byte offsets of every buffer.
struct Plan {
    size_t ncell = 0;
    int nlev = 0;
    LevelDims lev[kMaxLevels];
    int m = 0;
    size_t esz = 8;
    int N = 0, restart = 30, ntiles = 0;
    BlobGeom geom{};
    size_t off_grid[9]{};
    size_t off_lvl[kMaxLevels][5]{};
    size_t off_cinv[4]{};
    size_t off_part = 0, part_cap = 0;
    size_t off_sc = 0, off_gs = 0, off_dsc = 0;
    size_t off_q = 0, off_kappa = 0, off_base = 0, off_wts = 0, off_tile = 0, off_counts = 0, off_offsets = 0,
           off_cursor = 0, off_perm = 0;
    // spread contribution lists: per-tile counts and offsets, touched cells, entries
    size_t off_sp_cnt = 0, off_sp_off = 0, off_tcell = 0, off_tptr = 0, off_tblob = 0, off_tw = 0;
    // flexible-GMRES basis of the block solvers (handles that use them)
    size_t off_fg = 0, fg_size = 0;
    // handle-owned learned preconditioner: network state and room for the CSR of W
    size_t off_net = 0, off_lrn = 0, lrn_size = 0;
    size_t off_nv[12]{};
    size_t off_V = 0, off_H = 0, off_cs = 0, off_sn = 0, off_gv = 0, off_yv = 0;
    size_t total = 0;
};

// doubles between consecutive long vectors (grid part, blob part, padding)
size_t fg_stride(const Plan& P) { return (P.ncell + (size_t)P.N + 31) & ~(size_t)31; }

size_t fg_bytes(const Plan& P, int restart) {
    const size_t ld = (size_t)restart + 1;
    return (2 * (size_t)restart + 1) * fg_stride(P) * 8 + (ld * restart + 5 * ld + 8) * 8 + 256;
}

size_t net_bytes();
size_t learned_bytes(int N, long long nnz);

int make_plan(const blob_rd_params* p, Plan* P, std::string* why) {
    if (!p) {
        *why = "null params";
        return BLOB_RD_EINVAL;
    }
    if (p->nx < 8 || p->ny < 8 || p->nz < 8) {
        *why = "grid dims must be >= 8";
        return BLOB_RD_EINVAL;
    }
    if (!(p->h > 0.0) || !(p->D > 0.0)) {
        *why = "h and D must be positive";
        return BLOB_RD_EINVAL;
    }
    if (p->kernel_w != 3 && p->kernel_w != 4) {
        *why = "kernel_w must be 3 or 4";
        return BLOB_RD_EINVAL;
    }
    if (p->n_blobs < 0 || p->n_blobs > (1 << 26)) {
        *why = "n_blobs out of range";
        return BLOB_RD_EINVAL;
    }
    if (p->n_blobs > 0 && !p->q) {
        *why = "q is null";
        return BLOB_RD_EINVAL;
    }
    if (p->precision != BLOB_RD_FP64 && p->precision != BLOB_RD_MIXED) {
        *why = "precision must be FP64 (0) or MIXED (1)";
        return BLOB_RD_EINVAL;
    }
    if (p->boundary != BLOB_RD_BOUNDARY_PERIODIC && p->boundary != BLOB_RD_BOUNDARY_DIRICHLET) {
        *why = "boundary must be PERIODIC (0) or DIRICHLET (1)";
        return BLOB_RD_EINVAL;
    }
    if (!std::isfinite(p->boundary_value)) {
        *why = "boundary_value must be finite";
        return BLOB_RD_EINVAL;
    }
    const size_t ncell = (size_t)p->nx * p->ny * p->nz;
    if (ncell > (size_t)1 << 30) {
        *why = "grid too large";
        return BLOB_RD_EINVAL;
    }
    P->ncell = ncell;
    P->nlev = level_dims(p->nx, p->ny, p->nz, P->lev);
    if (P->nlev < 2) {
        *why = "grid cannot be coarsened";
        return BLOB_RD_EINVAL;
    }
    for (int l = 0; l < P->nlev; ++l) P->lev[l].h = p->h * (double)(1 << l);
    const LevelDims& C = P->lev[P->nlev - 1];
    P->m = C.nx * C.ny * C.nz;
    if (P->m > kMaxCoarse) {
        *why = "coarsest multigrid level exceeds 512 cells (dims must be 2^k times a small factor)";
        return BLOB_RD_EINVAL;
    }
    const int tx = tile_edge(p->nx), ty = tile_edge(p->ny), tz = tile_edge(p->nz);
    if (tx < 0 || ty < 0 || tz < 0) {
        *why = "each grid dim needs a divisor between 3 and 8";
        return BLOB_RD_EINVAL;
    }
    P->geom = BlobGeom{p->nx, p->ny, p->nz, tx, ty, tz, p->nx / tx, p->ny / ty, p->nz / tz, p->h, p->kernel_w};
    P->ntiles = P->geom.ntx * P->geom.nty * P->geom.ntz;
    P->esz = p->precision == BLOB_RD_MIXED ? 4 : 8;
    P->N = (int)p->n_blobs;
    P->restart = p->gmres_restart > 0 ? p->gmres_restart : 30;
    if (P->restart > 200) {
        *why = "gmres_restart must be <= 200";
        return BLOB_RD_EINVAL;
    }
    size_t o = 0;
    auto take = [&](size_t bytes) {
        size_t r = o;
        o = align_up(o + bytes);
        return r;
    };
    for (int i = 0; i < 9; ++i) P->off_grid[i] = take(ncell * 8);
    for (int l = 0; l < P->nlev - 1; ++l) {
        const size_t half = (size_t)P->lev[l].hx * P->lev[l].ny * P->lev[l].nz;
        // u0, u1, f0, f1 and the red residual r0 (the black residual is never stored)
        for (int k = 0; k < 5; ++k) P->off_lvl[l][k] = take(half * P->esz);
    }
    P->off_lvl[P->nlev - 1][0] = take((size_t)P->m * P->esz);  // coarsest u (natural)
    P->off_lvl[P->nlev - 1][2] = take((size_t)P->m * P->esz);  // coarsest f (natural)
    for (int k = 0; k < 4; ++k) P->off_cinv[k] = take((size_t)P->m * P->m * 8);
    P->part_cap = nblocks(ncell) + 64;
    P->off_part = take(P->part_cap * 3 * 8);
    P->off_sc = take(sizeof(Scalars));
    P->off_gs = take(sizeof(GmresScalars));
    P->off_dsc = take(64 * 8);
    const size_t N = (size_t)std::max(P->N, 1);
    P->off_q = take(N * 3 * 8);
    P->off_kappa = take(N * 8);
    P->off_base = take(N * 3 * 4);
    P->off_wts = take(N * 12 * 8);
    P->off_tile = take(N * 4);
    P->off_counts = take((size_t)P->ntiles * 4);
    P->off_offsets = take(((size_t)P->ntiles + 1) * 4);
    P->off_cursor = take((size_t)P->ntiles * 4);
    P->off_perm = take(N * 4);
    P->off_sp_cnt = take((size_t)P->ntiles * 2 * 4);
    P->off_sp_off = take(((size_t)P->ntiles + 1) * 2 * 4);
    P->off_tcell = take(N * 64 * 4);
    P->off_tptr = take((N * 64 + 1) * 4);
    P->off_tblob = take(N * 64 * 4);
    P->off_tw = take(N * 64 * 8);
    for (int k = 0; k < 12; ++k) P->off_nv[k] = take(N * 8);
    const size_t m = (size_t)P->restart;
    P->off_V = take((m + 1) * N * 8);
    P->off_H = take((m + 1) * m * 8);
    P->off_cs = take(m * 8);
    P->off_sn = take(m * 8);
    P->off_gv = take((m + 1) * 8);
    P->off_yv = take(m * 8);
    if (p->saddle_solver != BLOB_RD_SOLVER_SCHUR) {
        if (p->saddle_solver != BLOB_RD_SOLVER_BLOCK && p->saddle_solver != BLOB_RD_SOLVER_BLOCK_LEARNED) {
            *why = "unknown saddle_solver";
            return BLOB_RD_EINVAL;
        }
        P->fg_size = fg_bytes(*P, P->restart);
        P->off_fg = take(P->fg_size);
    }
    if ((p->schur_precond == BLOB_RD_PRECOND_LEARNED || p->saddle_solver == BLOB_RD_SOLVER_BLOCK_LEARNED) &&
        p->boundary == BLOB_RD_BOUNDARY_PERIODIC && P->N > 0) {
        P->off_net = take(net_bytes());
        P->lrn_size = learned_bytes(P->N, (long long)P->N * BLOB_RD_LEARNED_ROW_CAP);
        P->off_lrn = take(P->lrn_size);
    }
    P->total = o + 256;
    return 0;
}

// Dense (pseudo-)inverse of the coarsest operator alpha I - D L_H (row-major m x m).
// Periodic with alpha = 0 it returns (A + e e^T/m)^{-1} - e e^T/m, the pseudo-inverse
// on mean-zero vectors. In a box with fixed faces (box) a neighbour beyond a face is
// the ghost -u, which adds s to the diagonal; the operator is then invertible for
// every alpha >= 0. LU with partial pivoting, then column-wise solves.
std::vector<double> coarse_inverse(const LevelDims& C, double D, double alpha, bool box) {
    const int nx = C.nx, ny = C.ny, nz = C.nz, m = nx * ny * nz;
    const double s = D / (C.h * C.h);
    std::vector<double> A((size_t)m * m, 0.0);
    auto id = [&](int x, int y, int z) {
        if (box && (x < 0 || x >= nx || y < 0 || y >= ny || z < 0 || z >= nz)) return -1;
        x = (x + nx) % nx;
        y = (y + ny) % ny;
        z = (z + nz) % nz;
        return (z * ny + y) * nx + x;
    };
    for (int z = 0; z < nz; ++z)
        for (int y = 0; y < ny; ++y)
            for (int x = 0; x < nx; ++x) {
                const int r = id(x, y, z);
                A[(size_t)r * m + r] += alpha + 6.0 * s;
                const int nb[6] = {id(x - 1, y, z), id(x + 1, y, z), id(x, y - 1, z),
                                   id(x, y + 1, z), id(x, y, z - 1), id(x, y, z + 1)};
                for (int k = 0; k < 6; ++k) {
                    if (nb[k] < 0) A[(size_t)r * m + r] += s;  // ghost -u beyond a face
                    else A[(size_t)r * m + nb[k]] -= s;
                }
            }
    const bool sing = alpha == 0.0 && !box;
    const double e = 1.0 / m;
    if (sing)
        for (auto& v : A) v += e;
    std::vector<int> piv(m);
    for (int k = 0; k < m; ++k) {
        int pr = k;
        for (int i = k + 1; i < m; ++i)
            if (std::fabs(A[(size_t)i * m + k]) > std::fabs(A[(size_t)pr * m + k])) pr = i;
        piv[k] = pr;
        if (pr != k)
            for (int j = 0; j < m; ++j) std::swap(A[(size_t)k * m + j], A[(size_t)pr * m + j]);
        const double d = A[(size_t)k * m + k];
        if (d == 0.0) throw Err(BLOB_RD_ESINGULAR, "singular coarsest operator");
        for (int i = k + 1; i < m; ++i) {
            const double l = A[(size_t)i * m + k] / d;
            A[(size_t)i * m + k] = l;
            for (int j = k + 1; j < m; ++j) A[(size_t)i * m + j] -= l * A[(size_t)k * m + j];
        }
    }
    std::vector<double> inv((size_t)m * m);
    std::vector<double> col(m);
    for (int c = 0; c < m; ++c) {
        std::fill(col.begin(), col.end(), 0.0);
        col[c] = 1.0;
        for (int k = 0; k < m; ++k)
            if (piv[k] != k) std::swap(col[k], col[piv[k]]);
        for (int i = 0; i < m; ++i)
            for (int j = 0; j < i; ++j) col[i] -= A[(size_t)i * m + j] * col[j];
        for (int i = m - 1; i >= 0; --i) {
            for (int j = i + 1; j < m; ++j) col[i] -= A[(size_t)i * m + j] * col[j];
            col[i] /= A[(size_t)i * m + i];
        }
        for (int r = 0; r < m; ++r) inv[(size_t)r * m + c] = col[r] - (sing ? e : 0.0);
    }
    return inv;
}

}  // namespace

// ---------------------------------------------------------------------------
// The flexible-GMRES basis of blob_rd_solve_absorbing_fgmres_noalloc: a device array
// of the library (one per GPU in each process, held until the process ends), for
// callers that cannot allocate device memory. Host code never passes `scratch`
// itself to a kernel: it uses the device address taken once per device.
static __device__ __align__(256) unsigned char scratch[BLOB_RD_NOALLOC_BYTES];

namespace {

struct ScratchSlot {
    char* ptr = nullptr;
    std::mutex use;  // one no-alloc solve at a time on this GPU in this process
};
std::mutex g_scratch_m;
std::map<int, ScratchSlot> g_scratch;

// The current device's scratch slot; its address is taken on first use on that device.
ScratchSlot& scratch_slot() {
    int dev = 0;
    HIPCHK(hipGetDevice(&dev));
    std::lock_guard<std::mutex> lk(g_scratch_m);
    ScratchSlot& s = g_scratch[dev];
    if (!s.ptr) {
        void* p = nullptr;
        HIPCHK(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
        if (!p) throw Err(BLOB_RD_EDEVICE, "no device address for the no-alloc scratch");
        s.ptr = static_cast<char*>(p);
    }
    return s;
}

}  // namespace

struct BatchServer;

struct blob_rd {
    Plan P;
    blob_rd_params prm{};
    hipStream_t st = nullptr;
    char* ws = nullptr;
    double sum_kappa = 0.0;
    bool has_kappa = false;
    double cinv_alpha[4];
    int cinv_used = 0;
    int cinv_next = 0;
    // host mirrors (pinned)
    Scalars* hsc = nullptr;
    GmresScalars* hgs = nullptr;
    double* hbuf = nullptr;
    std::string err;
    // counters for stats of the current call
    int vcycles = 0;
    double alg_bytes = 0.0;
    int inner_iters = 0;
    int last_iters[4] = {0, 0, 0, 0};  // CG iterations of the previous solve per (blobs, alpha == 0)
    int tail_level[2] = {1 << 20, 1 << 20};  // first level of the LDS tail for FP32 / FP64 (>= nlev-1: none)
    // Work-group size per (level, multigrid kernel): Gauss-Seidel, residual, restriction,
    // prolongation. kBlock until blob_rd_autotune picks others.
    int bs[kMaxLevels][4];
    // CG iteration pairs captured as HIP graphs, keyed by (precision, blobs, alpha).
    struct GraphEntry {
        int esz;
        bool blobs;
        double alpha;
        hipGraphExec_t exec;
        double bytes_per_iter;
    };
    std::vector<GraphEntry> graphs;
    // block-FGMRES iterations captured as HIP graphs, one per basis index j and
    // configuration (basis workspace, alpha, preconditioner options), with the
    // counters one replay adds
    struct FgGraph {
        const char* ws;
        int j, esz, kind, m, n, restart, group;
        double alpha;
        bool fuse, learned;
        hipGraphExec_t exec;
        double bytes;
        int vcycles, inner, fallback;
    };
    std::vector<FgGraph> fg_graphs;
    bool fg_capture = true;  // off for calls that must not allocate
    hipStream_t cap_stream = nullptr;
    bool use_graphs = true;
    bool relax = true;  // relaxed inner tolerances in the Schur GMRES
    bool blocked = true;  // temporally blocked launches on the coarser per-level levels
    bool reorth_always = false;  // the block FGMRES re-orthogonalises every new basis vector
    // block FGMRES steps issued ahead of the host's reads: 0 never, 1 when the contraction says
    // the step in flight will not converge, 2 always (every converging step has one behind it)
    int fg_ahead = 1;
    // learned Schur preconditioner (CSR of W in a caller-provided buffer)
    struct Learned {
        bool ready = false;
        bool bad = false;      // non-finite entries: never used
        long long nnz = 0;
        int* rowptr = nullptr;
        int* col = nullptr;
        int* rowidx = nullptr;
        double* val = nullptr;
        float* dg = nullptr;
        float* nu = nullptr;  // per blob: other blobs within rc / 2 (a network input)
        PairGeom pg{};
    } lrn;
    int fallback = 0;
    // Fourier coarse level of the Schur preconditioner (in a caller-owned buffer): the basis Z,
    // M Z, E^{-1} = (Z^T M Z)^{-1} and the two folded into it (Z E^{-1}, M Z E^{-1}) for the
    // alpha it was built for, plus apply scratch
    struct Coarse {
        bool ready = false;
        double alpha = 0.0;
        int K = 0;
        int* modes = nullptr;
        double* Z = nullptr;
        double* MZ = nullptr;
        double* ZE = nullptr;   // Z E^{-1}
        double* MZE = nullptr;  // M Z E^{-1}
        double* Einv = nullptr;
        double* E = nullptr;
        double* r2 = nullptr;
        double* w = nullptr;
        double* part = nullptr;  // (K + 1) x (row chunks) partial dot products
        double* a = nullptr;
        double w0 = 0.0;  // scale of W without the learned part: 4 pi a0 D (eq. Schur_diagonal)
    } crs;
    // network owned by the handle (handles created for the learned preconditioner): its state
    // and W live in the handle's workspace; own_w says W was built from it
    blob_rd_net* own_net = nullptr;
    bool own_w = false;
    int ntouched = 0;  // cells with a nonzero spread weight (length of the contribution lists)
    // box with the concentration held at cb on its faces (solves work on u = c - cb)
    bool box = false;
    double cb = 0.0;
    // lock-step batch executor this handle currently belongs to (null: solo); batch_v: its
    // block-FGMRES V-cycles run in the executor's batched V-cycle rounds (batch_ev orders them
    // after the handle's own work)
    BatchServer* batch = nullptr;
    int batch_slot = -1;
    bool batch_v = false;
    hipEvent_t batch_ev = nullptr;
    // block FGMRES: the two steps in flight copy their residual estimates to hbuf[8..11]
    hipEvent_t fg_ev[2] = {nullptr, nullptr};
    // this device's no-alloc scratch (device address of `scratch`, taken at create)
    ScratchSlot* noalloc = nullptr;

    template <typename T>
    T* at(size_t off) const {
        return reinterpret_cast<T*>(ws + off);
    }
    double* grid(int i) const { return at<double>(P.off_grid[i]); }
    Scalars* sc() const { return at<Scalars>(P.off_sc); }
    GmresScalars* gs() const { return at<GmresScalars>(P.off_gs); }
    double* part() const { return at<double>(P.off_part); }
    double* dsc() const { return at<double>(P.off_dsc); }
    double* nv(int k) const { return at<double>(P.off_nv[k]); }
    double inv_h3() const { return 1.0 / (prm.h * prm.h * prm.h); }
};

namespace {

// G_S holds the right-hand side of an absorbing time step for the whole solve
enum GridBuf { G_R = 0, G_P = 1, G_Q = 2, G_U = 3, G_G = 4, G_T1 = 5, G_T2 = 6, G_P2 = 7, G_S = 8 };

__global__ void k_sc_init(Scalars* sc, int project, double inv_ncell, double eBe_inv, double rtol2, double abs2,
                          int xzero) {
    sc->xzero = xzero;
    sc->rz = 0.0;
    sc->pq = 0.0;
    sc->alpha = 0.0;
    sc->beta = 0.0;
    sc->rr = 0.0;
    sc->rsum = 0.0;
    sc->qsum = 0.0;
    sc->tol2 = rtol2;
    sc->shift = 0.0;
    sc->mean_r = 0.0;
    sc->mean_next = 0.0;
    sc->inv_ncell = inv_ncell;
    sc->eBe_inv = eBe_inv;
    sc->rr0 = abs2;
    sc->gg = 0.0;
    sc->done = 0;
    sc->iters = 0;
    sc->project = project;
    sc->status = 0;
}

void sync_read(blob_rd* H, void* host, const void* dev, size_t bytes) {
    HIPCHK(hipMemcpyAsync(host, dev, bytes, hipMemcpyDeviceToHost, H->st));
    HIPCHK(hipStreamSynchronize(H->st));
}

const double* select_cinv(blob_rd* H, double alpha) {
    for (int k = 0; k < H->cinv_used; ++k)
        if (H->cinv_alpha[k] == alpha) return H->at<double>(H->P.off_cinv[k]);
    const int slot = H->cinv_next;
    H->cinv_next = (H->cinv_next + 1) % 4;
    if (H->cinv_used < 4) {
        ++H->cinv_used;
    } else {
        // graphs captured for the evicted alpha point at this slot: drop them
        HIPCHK(hipStreamSynchronize(H->st));
        const double old = H->cinv_alpha[slot];
        for (size_t i = 0; i < H->graphs.size();) {
            if (H->graphs[i].alpha == old) {
                (void)hipGraphExecDestroy(H->graphs[i].exec);
                H->graphs.erase(H->graphs.begin() + i);
            } else {
                ++i;
            }
        }
        for (size_t i = 0; i < H->fg_graphs.size();) {
            if (H->fg_graphs[i].alpha == old) {
                (void)hipGraphExecDestroy(H->fg_graphs[i].exec);
                H->fg_graphs.erase(H->fg_graphs.begin() + i);
            } else {
                ++i;
            }
        }
    }
    H->cinv_alpha[slot] = alpha;
    std::vector<double> inv = coarse_inverse(H->P.lev[H->P.nlev - 1], H->prm.D, alpha, H->box);
    double* dst = H->at<double>(H->P.off_cinv[slot]);
    HIPCHK(hipMemcpyAsync(dst, inv.data(), inv.size() * 8, hipMemcpyHostToDevice, H->st));
    HIPCHK(hipStreamSynchronize(H->st));
    return dst;
}

// One V(2,2) cycle for alpha I - D L applied to the FP64 natural vector r
// (mean_r removed when the scalars say so); the result is left in level 0's
// u arrays (split layout).
// First level of the single-work-group LDS tail: the coarsest levels whose
// u, f, r arrays fit the LDS budget together.
int tail_start(const Plan& P, size_t esz, size_t budget) {
    const int L = P.nlev - 1;
    int t = L;  // never used as is: the tail always includes one smoothing level
    size_t bytes = 2 * (size_t)P.m * esz + 64;
    for (int l = L - 1; l >= 0; --l) {
        const size_t c = (size_t)P.lev[l].nx * P.lev[l].ny * P.lev[l].nz;
        const size_t add = 3 * ((c * esz + 15) & ~(size_t)15);
        if (bytes + add > budget || c > 16 * 1024) break;
        bytes += add;
        t = l;
    }
    return t;
}

template <typename T>
TailDesc make_tail(const blob_rd* H, int t, double alpha) {
    const Plan& P = H->P;
    TailDesc d{};
    const int L = P.nlev - 1;
    d.nlev = L - t + 1;
    d.m = P.m;
    unsigned o = 0;
    auto take = [&](size_t n) {
        unsigned r = o;
        o += (unsigned)((n * sizeof(T) + 15) & ~(size_t)15);
        return r;
    };
    for (int k = 0; k < d.nlev; ++k) {
        const LevelDims& ld = P.lev[t + k];
        d.nx[k] = ld.nx;
        d.ny[k] = ld.ny;
        d.nz[k] = ld.nz;
        const double s = H->prm.D / (ld.h * ld.h);
        d.s[k] = s;
        d.diag[k] = alpha + 6.0 * s;
        d.inv_diag[k] = 1.0 / (alpha + 6.0 * s);
        const size_t n = (size_t)ld.nx * ld.ny * ld.nz;
        d.off_u[k] = take(n);
        d.off_f[k] = take(n);
        d.off_r[k] = (k + 1 < d.nlev) ? take(n) : 0;
    }
    d.lds_bytes = o;
    return d;
}

// Algorithmic bytes per fine cell of a level, in units of the level's element
// size (each input read once, each output written once): three half-sweeps,
// the red residual, its restriction and the coarse f and u on the way down;
// the red-cell correction (the black cells are overwritten by the next black
// half-sweep, which does not read them) and four half-sweeps on the way up.
constexpr double kPreRestrictBytes = 3 * 1.5 + 2.0 + 0.5 + 0.1875;
constexpr double kProlongPostBytes = 1.125 + 4 * 1.5;
// temporally blocked levels: red u and f in, pre-smoothed red and coarse f, u out;
// coarse u, pre-smoothed red and f in, both colours out
constexpr double kBlockedDownBytes = 0.5 + 1.0 + 0.5 + 0.1875;
constexpr double kBlockedUpBytes = 0.125 + 0.5 + 1.0 + 1.0;

// alpha I - D L has a null space (the constant) only on the periodic grid with alpha = 0
bool singular(const blob_rd* H, double alpha) { return alpha == 0.0 && !H->box; }

// Diagonal and inverse diagonal of level l of a box with fixed faces, per number of
// faces a cell touches.
void box_coefs(const blob_rd* H, int l, double alpha, BoxCoef* diag, BoxCoef* inv) {
    const LevelDims& d = H->P.lev[l];
    const double s = H->prm.D / (d.h * d.h);
    for (int f = 0; f < 4; ++f) {
        const double v = alpha + s * (6.0 + f);
        if (diag) diag->v[f] = v;
        if (inv) inv->v[f] = 1.0 / v;
    }
}

// The V-cycle of vcycle() below for the box operator alpha I - D L_0: the same
// steps and order with the box kernels, per-level launches down to the first
// level of the LDS tail (then the box tail kernel) or to the coarsest level (the
// dense box inverse); no temporally blocked levels.
template <typename T>
void vcycle_box(blob_rd* H, double alpha, const double* r, const Scalars* sc, const double* cinv, bool entered) {
    const Plan& P = H->P;
    const int L = P.nlev - 1;
    const int t = std::min(H->tail_level[sizeof(T) == 4 ? 0 : 1], L);
    hipStream_t st = H->st;
    auto lv = [&](int l, int k) { return H->at<T>(P.off_lvl[l][k]); };  // 0 u0, 1 u1, 2 f0, 3 f1, 4 r0 (red)
    BoxCoef dg[kMaxLevels], inv[kMaxLevels];
    for (int l = 0; l <= L; ++l) box_coefs(H, l, alpha, &dg[l], &inv[l]);
    if (!entered) {
        const LevelDims& d = P.lev[0];
        launch_enter_box<T>(st, r, lv(0, 2), lv(0, 3), lv(0, 0), d.nx, d.ny, d.nz, inv[0], sc);
        H->alg_bytes += (double)P.ncell * (8 + P.esz * 1.5);
    }
    for (int l = 0; l < t; ++l) {
        const LevelDims& d = P.lev[l];
        const double s = H->prm.D / (d.h * d.h);
        launch_gs_box<T>(st, lv(l, 1), lv(l, 0), lv(l, 3), d.nx, d.ny, d.nz, 1, s, inv[l], sc);
        launch_gs_box<T>(st, lv(l, 0), lv(l, 1), lv(l, 2), d.nx, d.ny, d.nz, 0, s, inv[l], sc);
        launch_gs_box<T>(st, lv(l, 1), lv(l, 0), lv(l, 3), d.nx, d.ny, d.nz, 1, s, inv[l], sc);
        launch_resid_red_box<T>(st, lv(l, 0), lv(l, 1), lv(l, 2), lv(l, 4), d.nx, d.ny, d.nz, s, dg[l], sc);
        if (l + 1 == L)
            launch_restrict_box<T>(st, lv(l, 4), d.nx, d.ny, d.nz, lv(L, 2), nullptr, nullptr, 1, inv[L], sc);
        else
            launch_restrict_box<T>(st, lv(l, 4), d.nx, d.ny, d.nz, lv(l + 1, 2), lv(l + 1, 3), lv(l + 1, 0), 0,
                                   inv[l + 1], sc);
        H->alg_bytes += (double)P.ncell / (1 << (3 * l)) * P.esz * kPreRestrictBytes;
    }
    if (t < L) launch_tail_box<T>(st, lv(t, 2), lv(t, 3), lv(t, 0), lv(t, 1), make_tail<T>(H, t, alpha), cinv, sc);
    else launch_coarse<T>(st, lv(L, 2), lv(L, 0), cinv, P.m, sc);
    for (int l = t - 1; l >= 0; --l) {
        const LevelDims& d = P.lev[l];
        const double s = H->prm.D / (d.h * d.h);
        const int cnat = (l + 1 == L);
        launch_prolong_red_box<T>(st, lv(l + 1, 0), cnat ? nullptr : lv(l + 1, 1), cnat, lv(l, 0), d.nx, d.ny, d.nz,
                                  sc);
        launch_gs_box<T>(st, lv(l, 1), lv(l, 0), lv(l, 3), d.nx, d.ny, d.nz, 1, s, inv[l], sc);
        launch_gs_box<T>(st, lv(l, 0), lv(l, 1), lv(l, 2), d.nx, d.ny, d.nz, 0, s, inv[l], sc);
        launch_gs_box<T>(st, lv(l, 1), lv(l, 0), lv(l, 3), d.nx, d.ny, d.nz, 1, s, inv[l], sc);
        launch_gs_box<T>(st, lv(l, 0), lv(l, 1), lv(l, 2), d.nx, d.ny, d.nz, 0, s, inv[l], sc);
        H->alg_bytes += (double)P.ncell / (1 << (3 * l)) * P.esz * kProlongPostBytes;
    }
    H->vcycles += 1;
}

// entered: level 0's f and first red sweep were already written (fused CG
// update). dot_q (with a non-null sc): fuse the CG dots (sum z, z.r, z.q) into
// the closing red half-sweep of level 0 when that level has its own launches;
// returns the number of partials written to H->part(), 0 when not fused.
template <typename T>
unsigned vcycle(blob_rd* H, double alpha, const double* r, const Scalars* sc, const double* cinv,
                bool entered = false, const double* dot_q = nullptr, bool from_f = false) {
    if (H->box) {
        vcycle_box<T>(H, alpha, r, sc, cinv, entered);
        return 0;
    }
    const Plan& P = H->P;
    const int L = P.nlev - 1;
    hipStream_t st = H->st;
    auto lv = [&](int l, int k) { return H->at<T>(P.off_lvl[l][k]); };  // 0 u0, 1 u1, 2 f0, 3 f1, 4 r0 (red)
    const double D = H->prm.D;
    const int t = H->tail_level[sizeof(T) == 4 ? 0 : 1];
    unsigned ndots = 0;
    // closing red half-sweep of level l (with the CG dots on level 0 when asked;
    // that launch keeps the default work-group size, so its partial sums, and
    // with them every result, do not depend on the tuning table)
    auto last_red = [&](int l, double s, double diag, const int* b) {
        const LevelDims& d = P.lev[l];
        if (l == 0 && dot_q && sc)
            ndots = launch_gs_dots<T>(st, lv(0, 0), lv(0, 1), lv(0, 2), d.hx, d.ny, d.nz, s, 1.0 / diag, r, dot_q,
                                      H->part(), sc, kBlock);
        if (!(l == 0 && ndots))
            launch_gs<T>(st, lv(l, 0), lv(l, 1), lv(l, 2), d.hx, d.ny, d.nz, 0, s, 1.0 / diag, sc, b[0]);
    };
    // opening black half-sweep of level l; with from_f, level 0's red u is not stored by the
    // entry and the sweep takes it as f_red / diag (it keeps the default work-group size)
    auto first_black = [&](int l, double s, double diag, const int* b) {
        const LevelDims& d = P.lev[l];
        if (l == 0 && from_f &&
            launch_gs_from_f<T>(st, lv(0, 1), lv(0, 2), lv(0, 3), d.hx, d.ny, d.nz, 1, s, 1.0 / diag, sc))
            return;
        if (l == 0 && from_f) throw Err(BLOB_RD_EDEVICE, "V-cycle entry without a stored red sweep");
        launch_gs<T>(st, lv(l, 1), lv(l, 0), lv(l, 3), d.hx, d.ny, d.nz, 1, s, 1.0 / diag, sc, b[0]);
    };
    if (!entered) {
        // with from_f the first red sweep is not stored: the opening black sweep forms it
        const LevelDims& d = P.lev[0];
        const double s = D / (d.h * d.h);
        launch_enter<T>(st, r, lv(0, 2), lv(0, 3), from_f ? nullptr : lv(0, 0), d.nx, d.ny, d.nz,
                        1.0 / (alpha + 6.0 * s), sc);
        H->alg_bytes += (double)P.ncell * (8 + P.esz * (from_f ? 1.0 : 1.5));
    }
    // levels below the finest whose pre- and post-smoothing run temporally blocked:
    // those of at most 64^3 cells, where a launch costs more than the level's bytes
    // (on larger levels the recomputed halos cost more than the launches they save)
    auto blocked = [&](int l) {
        const LevelDims& d = P.lev[l];
        return H->blocked && l >= 1 && d.nx % 8 == 0 && d.ny % 8 == 0 && d.nz % 8 == 0 &&
               (size_t)d.nx * d.ny * d.nz <= (size_t)64 * 64 * 64;
    };
    if (t < L) {
        for (int l = 0; l < t; ++l) {
            const LevelDims& d = P.lev[l];
            const double s = D / (d.h * d.h), diag = alpha + 6.0 * s;
            if (blocked(l)) {
                const LevelDims& c = P.lev[l + 1];
                launch_down<T>(st, lv(l, 0), lv(l, 2), lv(l, 3), lv(l, 4), d.nx, d.ny, d.nz, s, diag, lv(l + 1, 2),
                               lv(l + 1, 3), lv(l + 1, 0), 1.0 / (alpha + 6.0 * (D / (c.h * c.h))), sc);
                H->alg_bytes += (double)P.ncell / (1 << (3 * l)) * P.esz * kBlockedDownBytes;
                continue;
            }
            const int* b = H->bs[l];
            first_black(l, s, diag, b);
            launch_gs<T>(st, lv(l, 0), lv(l, 1), lv(l, 2), d.hx, d.ny, d.nz, 0, s, 1.0 / diag, sc, b[0]);
            launch_gs<T>(st, lv(l, 1), lv(l, 0), lv(l, 3), d.hx, d.ny, d.nz, 1, s, 1.0 / diag, sc, b[0]);
            launch_resid_red<T>(st, lv(l, 0), lv(l, 1), lv(l, 2), lv(l, 4), d.hx, d.ny, d.nz, s, diag, sc, b[1]);
            const LevelDims& c = P.lev[l + 1];
            const double sc_ = D / (c.h * c.h);
            launch_restrict<T>(st, lv(l, 4), d.nx, d.ny, d.nz, lv(l + 1, 2), lv(l + 1, 3), lv(l + 1, 0), 0,
                               1.0 / (alpha + 6.0 * sc_), sc, b[2]);
            H->alg_bytes += (double)P.ncell / (1 << (3 * l)) * P.esz * kPreRestrictBytes;
        }
        const TailDesc td = make_tail<T>(H, t, alpha);
        launch_tail<T>(st, lv(t, 2), lv(t, 3), lv(t, 0), lv(t, 1), td, cinv, sc);
        for (int l = t - 1; l >= 0; --l) {
            const LevelDims& d = P.lev[l];
            const double s = D / (d.h * d.h), diag = alpha + 6.0 * s;
            if (blocked(l)) {
                launch_up<T>(st, lv(l + 1, 0), lv(l + 1, 1), lv(l, 4), lv(l, 2), lv(l, 3), lv(l, 0), lv(l, 1), d.nx,
                             d.ny, d.nz, s, diag, sc);
                H->alg_bytes += (double)P.ncell / (1 << (3 * l)) * P.esz * kBlockedUpBytes;
                continue;
            }
            const int* b = H->bs[l];
            launch_prolong<T>(st, lv(l + 1, 0), lv(l + 1, 1), 0, lv(l, 0), lv(l, 1), d.nx, d.ny, d.nz, sc, b[3]);
            launch_gs<T>(st, lv(l, 1), lv(l, 0), lv(l, 3), d.hx, d.ny, d.nz, 1, s, 1.0 / diag, sc, b[0]);
            launch_gs<T>(st, lv(l, 0), lv(l, 1), lv(l, 2), d.hx, d.ny, d.nz, 0, s, 1.0 / diag, sc, b[0]);
            launch_gs<T>(st, lv(l, 1), lv(l, 0), lv(l, 3), d.hx, d.ny, d.nz, 1, s, 1.0 / diag, sc, b[0]);
            last_red(l, s, diag, b);
            H->alg_bytes += (double)P.ncell / (1 << (3 * l)) * P.esz * kProlongPostBytes;
        }
        H->vcycles += 1;
        return ndots;
    }
    for (int l = 0; l < L; ++l) {
        const LevelDims& d = P.lev[l];
        const double s = D / (d.h * d.h), diag = alpha + 6.0 * s;
        const int* b = H->bs[l];
        first_black(l, s, diag, b);
        launch_gs<T>(st, lv(l, 0), lv(l, 1), lv(l, 2), d.hx, d.ny, d.nz, 0, s, 1.0 / diag, sc, b[0]);
        launch_gs<T>(st, lv(l, 1), lv(l, 0), lv(l, 3), d.hx, d.ny, d.nz, 1, s, 1.0 / diag, sc, b[0]);
        launch_resid_red<T>(st, lv(l, 0), lv(l, 1), lv(l, 2), lv(l, 4), d.hx, d.ny, d.nz, s, diag, sc, b[1]);
        const int cnat = (l + 1 == L);
        const LevelDims& c = P.lev[l + 1];
        const double sc_ = D / (c.h * c.h);
        if (cnat)
            launch_restrict<T>(st, lv(l, 4), d.nx, d.ny, d.nz, lv(L, 2), nullptr, nullptr, 1, 0.0, sc, b[2]);
        else
            launch_restrict<T>(st, lv(l, 4), d.nx, d.ny, d.nz, lv(l + 1, 2), lv(l + 1, 3), lv(l + 1, 0), 0,
                               1.0 / (alpha + 6.0 * sc_), sc, b[2]);
        H->alg_bytes += (double)P.ncell / (1 << (3 * l)) * P.esz * kPreRestrictBytes;
    }
    launch_coarse<T>(st, lv(L, 2), lv(L, 0), cinv, P.m, sc);
    for (int l = L - 1; l >= 0; --l) {
        const LevelDims& d = P.lev[l];
        const double s = D / (d.h * d.h), diag = alpha + 6.0 * s;
        const int cnat = (l + 1 == L);
        const int* b = H->bs[l];
        launch_prolong<T>(st, lv(l + 1, 0), cnat ? nullptr : lv(l + 1, 1), cnat, lv(l, 0), lv(l, 1), d.nx, d.ny, d.nz,
                          sc, b[3]);
        launch_gs<T>(st, lv(l, 1), lv(l, 0), lv(l, 3), d.hx, d.ny, d.nz, 1, s, 1.0 / diag, sc, b[0]);
        launch_gs<T>(st, lv(l, 0), lv(l, 1), lv(l, 2), d.hx, d.ny, d.nz, 0, s, 1.0 / diag, sc, b[0]);
        launch_gs<T>(st, lv(l, 1), lv(l, 0), lv(l, 3), d.hx, d.ny, d.nz, 1, s, 1.0 / diag, sc, b[0]);
        last_red(l, s, diag, b);
        H->alg_bytes += (double)P.ncell / (1 << (3 * l)) * P.esz * kProlongPostBytes;
    }
    H->vcycles += 1;
    return ndots;
}

template <typename T>
void precond_zdots(blob_rd* H, double alpha, const double* r, const double* q, const double* cinv,
                   bool entered = false) {
    unsigned np = vcycle<T>(H, alpha, r, H->sc(), cinv, entered, q);
    if (np) {
        H->alg_bytes += (double)H->P.ncell * 16;  // r, q read by the fused sweep
    } else {
        const LevelDims& d = H->P.lev[0];
        launch_zdots2<T>(H->st, H->at<T>(H->P.off_lvl[0][0]), H->at<T>(H->P.off_lvl[0][1]), r, q, d.nx, d.ny, d.nz,
                         H->part(), H->sc(), &np);
        H->alg_bytes += (double)H->P.ncell * (H->P.esz + 16);
    }
    launch_fin(H->st, FIN_BETA, H->part(), np, H->sc(), nullptr, nullptr, 0, 0.0);
}

// out = base_in + scale * S (lam + lam_shift) from the contribution lists: a
// dense pass (copy of base_in, or zeros without it; none when out aliases
// base_in) and one thread per touched cell. lam may be null (lam_shift only).
void spread_to(blob_rd* H, const double* lam, double lam_shift, const double* base_in, double* out, double scale,
               const Scalars* sc) {
    const Plan& P = H->P;
    if (base_in != out) {
        if (base_in) launch_nvec_copy_scale(H->st, base_in, out, (int)P.ncell, 1.0, 0.0);
        else launch_fill(H->st, out, P.ncell, 0.0);
    }
    launch_spread_sparse(H->st,
                         SpreadLists{H->ntouched, H->at<int>(P.off_tcell), H->at<int>(P.off_tptr),
                                     H->at<int>(P.off_tblob), H->at<double>(P.off_tw)},
                         SpreadMult{lam, nullptr, 0.0, lam_shift}, base_in, out, scale, sc);
}

// q += S kappa J p, with jx = J p and mu = kappa J p kept for the CG dots.
void blob_term(blob_rd* H, const double* p, double* q, const Scalars* sc) {
    const Plan& P = H->P;
    launch_interp(H->st, p, P.N, P.geom, H->at<int>(P.off_base), H->at<double>(P.off_wts), H->at<int>(P.off_perm),
                  H->nv(0), H->at<double>(P.off_kappa), H->nv(1), sc);
    spread_to(H, H->nv(1), 0.0, q, q, H->inv_h3(), sc);
}

// Batch executor hooks (defined with the executor below).
void batch_run_cg(blob_rd* H, double* x, int maxit, bool blobs, double alpha);

// Algorithmic bytes of one CG iteration inside the CG loop (update with the
// V-cycle entry, V-cycle with the fused dots).
double iteration_bytes(const blob_rd* H) {
    const Plan& P = H->P;
    const int L = P.nlev - 1;
    const int t = std::min(H->tail_level[P.esz == 4 ? 0 : 1], L);
    double b = (double)P.ncell * (P.esz + 16 + 16 + 48 + 1.5 * P.esz) + (double)P.ncell * 16;
    for (int l = 0; l < t; ++l) b += (double)P.ncell / (1 << (3 * l)) * P.esz * (kPreRestrictBytes + kProlongPostBytes);
    return b;
}

struct PcgResult {
    int iters = 0;
    int status = 0;
    bool converged = false;
    double rr = 0.0, gg = 0.0;
};

// CG on (alpha I - D L [+ S kappa J]) x = g. x_zero: start from x = 0 (x is
// overwritten). Stops at |r|^2 <= max(rtol^2 |g|^2, abs_tol^2).
template <typename T>
PcgResult pcg(blob_rd* H, bool with_blobs, double alpha, const double* g, double* x, bool x_zero, double rtol,
              double abs_tol, int maxit) {
    const Plan& P = H->P;
    hipStream_t st = H->st;
    double* r = H->grid(G_R);
    double* pbuf[2] = {H->grid(G_P), H->grid(G_P2)};
    int parity = 0;
    double* q = H->grid(G_Q);
    const LevelDims& d = P.lev[0];
    const double s = H->prm.D / (d.h * d.h);
    const int project = singular(H, alpha) ? 1 : 0;
    const bool blobs = with_blobs && P.N > 0 && H->has_kappa;
    BoxCoef binv;
    box_coefs(H, 0, alpha, nullptr, &binv);
    const double eBe = alpha * (double)P.ncell + H->sum_kappa * H->inv_h3();
    const double eBe_inv = (with_blobs && project && eBe > 0.0) ? 1.0 / eBe : 0.0;
    const double* cinv = select_cinv(H, alpha);
    hipLaunchKernelGGL(k_sc_init, dim3(1), dim3(1), 0, st, H->sc(), project, 1.0 / (double)P.ncell, eBe_inv,
                       rtol * rtol, abs_tol * abs_tol, x_zero ? 1 : 0);
    unsigned np = 0;
    if (x_zero) {
        // x = 0 is written by the first update (or below when no iteration runs)
        if (g == r) {
            launch_self_partials(st, g, P.ncell, H->part(), &np);
            H->alg_bytes += (double)P.ncell * 8;
        } else {
            launch_residual_from_q(st, g, nullptr, r, P.ncell, H->part(), &np);
            H->alg_bytes += (double)P.ncell * 16;
        }
    } else {
        launch_applyA_plain(st, x, q, alpha, s, d.nx, d.ny, d.nz, H->box);
        if (blobs) blob_term(H, x, q, nullptr);
        launch_residual_from_q(st, g, q, r, P.ncell, H->part(), &np);
        H->alg_bytes += (double)P.ncell * 40;
    }
    launch_fin(st, FIN_INIT, H->part(), np, H->sc(), nullptr, nullptr, 0, 0.0);
    precond_zdots<T>(H, alpha, r, q, cinv);
    int& hist = H->last_iters[(with_blobs ? 2 : 0) + project];
    int chunk = hist > 0 ? std::min(hist, maxit) : std::min(4, maxit);
    int done_iters = 0;
    PcgResult res;
    // One CG iteration; all scalars come from device memory, so the sequence
    // is identical from one iteration to the next apart from the p parity.
    auto iteration = [&](hipStream_t s_) {
        hipStream_t keep = H->st;
        H->st = s_;
        double* p = pbuf[0];
        (void)parity;
        launch_dir2<T>(s_, H->at<T>(P.off_lvl[0][0]), H->at<T>(P.off_lvl[0][1]), p, d.nx, d.ny, d.nz, H->sc());
        launch_applyA2(s_, p, q, alpha, s, d.nx, d.ny, d.nz, H->part(), H->sc(), &np, H->box);
        if (blobs) {
            blob_term(H, p, q, H->sc());
            launch_fin(s_, FIN_ALPHA, H->part(), np, H->sc(), H->nv(0), H->nv(1), P.N, H->inv_h3());
        } else {
            launch_fin(s_, FIN_ALPHA, H->part(), np, H->sc(), nullptr, nullptr, 0, 0.0);
        }
        launch_update2_enter<T>(s_, x, r, p, q, H->at<T>(P.off_lvl[0][2]), H->at<T>(P.off_lvl[0][3]),
                                H->at<T>(P.off_lvl[0][0]), d.nx, d.ny, d.nz, 1.0 / (alpha + 6.0 * s), H->part(),
                                H->sc(), &np, H->box ? &binv : nullptr);
        launch_fin(s_, FIN_UPDATE, H->part(), np, H->sc(), nullptr, nullptr, 0, 0.0);
        precond_zdots<T>(H, alpha, r, q, cinv, true);
        // direction (z, p r/w), stencil (p, q), update (x, r r/w, p, q) with the V-cycle entry (f, red u)
        H->alg_bytes += (double)P.ncell * (P.esz + 16 + 16 + 48 + 1.5 * P.esz);
        H->st = keep;
    };
    if (H->batch) {
        // The lock-step batch executor runs this solve's iterations in its
        // batched launches, together with the other instances' solves.
        HIPCHK(hipStreamSynchronize(st));
        batch_run_cg(H, x, maxit, blobs, alpha);
        sync_read(H, H->hsc, H->sc(), sizeof(Scalars));
        res.iters = H->hsc->iters;
        hist = res.iters;
        H->alg_bytes += iteration_bytes(H) * res.iters;
        H->vcycles += res.iters;
        res.status = H->hsc->status;
        res.rr = H->hsc->rr;
        res.gg = H->hsc->gg;
        res.converged = H->hsc->done && H->hsc->status == 0;
        if (x_zero && res.iters == 0) launch_fill(st, x, P.ncell, 0.0);
        return res;
    }
    blob_rd::GraphEntry* ge = nullptr;
    if (H->use_graphs && x == H->grid(G_U)) {
        for (auto& g : H->graphs)
            if (g.esz == (int)sizeof(T) && g.blobs == blobs && g.alpha == alpha) ge = &g;
        if (!ge) {
            if (!H->cap_stream) HIPCHK(hipStreamCreateWithFlags(&H->cap_stream, hipStreamNonBlocking));
            const double b0 = H->alg_bytes;
            const int v0 = H->vcycles;
            HIPCHK(hipStreamBeginCapture(H->cap_stream, hipStreamCaptureModeThreadLocal));
            iteration(H->cap_stream);
            iteration(H->cap_stream);
            hipGraph_t graph;
            HIPCHK(hipStreamEndCapture(H->cap_stream, &graph));
            hipGraphExec_t exec;
            HIPCHK(hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0));
            (void)hipGraphDestroy(graph);
            H->graphs.push_back({(int)sizeof(T), blobs, alpha, exec, 0.5 * (H->alg_bytes - b0)});
            ge = &H->graphs.back();
            H->alg_bytes = b0;
            H->vcycles = v0;
        }
    }
    for (;;) {
        if (ge) {
            for (int k = 0; k < chunk; k += 2) HIPCHK(hipGraphLaunch(ge->exec, st));
        } else {
            // an even number of iterations keeps the p parity aligned with the graphs
            chunk += chunk & 1;
            for (int k = 0; k < chunk; ++k) iteration(st);
        }
        sync_read(H, H->hsc, H->sc(), sizeof(Scalars));
        done_iters = H->hsc->iters;
        if (H->hsc->done || done_iters >= maxit) break;
        // predict the remaining iterations from the observed contraction
        const Scalars& hs = *H->hsc;
        chunk = 4;
        if (done_iters > 0 && hs.rr0 > 0.0 && hs.rr > 0.0 && hs.tol2 > 0.0 && hs.rr < hs.rr0) {
            const double rho = std::pow(hs.rr / hs.rr0, 0.5 / done_iters);
            const double rem = std::log(std::sqrt(hs.tol2 / hs.rr)) / std::log(rho);
            if (std::isfinite(rem)) chunk = (int)std::ceil(rem);
        }
        chunk = std::max(1, std::min(16, chunk));
        if (done_iters + chunk > maxit) chunk = maxit - done_iters;
    }
    res.iters = H->hsc->iters;
    hist = res.iters;
    if (ge) {
        H->alg_bytes += ge->bytes_per_iter * res.iters;
        H->vcycles += res.iters;
    }
    res.status = H->hsc->status;
    res.rr = H->hsc->rr;
    res.gg = H->hsc->gg;
    res.converged = H->hsc->done && H->hsc->status == 0;
    if (x_zero && res.iters == 0) launch_fill(st, x, P.ncell, 0.0);
    return res;
}

// True FP64 residual t = g - B x; returns |t| and |g|.
void true_residual(blob_rd* H, bool with_blobs, double alpha, const double* g, const double* x, double* t, double* rn,
                   double* gn) {
    const Plan& P = H->P;
    const LevelDims& d = P.lev[0];
    const double s = H->prm.D / (d.h * d.h);
    double* q = H->grid(G_Q);
    launch_applyA_plain(H->st, x, q, alpha, s, d.nx, d.ny, d.nz, H->box);
    if (with_blobs && P.N > 0 && H->has_kappa) blob_term(H, x, q, nullptr);
    unsigned np = 0;
    launch_residual_from_q(H->st, g, q, t, P.ncell, H->part(), &np);
    launch_reduce_parts(H->st, H->part(), np, 3, H->dsc());
    sync_read(H, H->hbuf, H->dsc(), 3 * 8);
    *rn = std::sqrt(H->hbuf[0]);
    *gn = std::sqrt(H->hbuf[2]);
    H->alg_bytes += (double)P.ncell * 40;
}

int default_maxit(blob_rd* H) { return H->prm.max_iter > 0 ? H->prm.max_iter : 1000; }
int inner_maxit(blob_rd* H) { return H->prm.inner_max_iter > 0 ? H->prm.inner_max_iter : 200; }

template <typename T>
int reactive_solve(blob_rd* H, double alpha, const double* g, double* c, blob_rd_stats* stt) {
    const double rtol = H->prm.rtol > 0.0 ? H->prm.rtol : 1e-8;
    int total = 0, refinements = 0;
    double rn = 0.0, gn = 1.0;
    bool ok = false;
    double* x = H->grid(G_U);
    launch_axpby(H->st, x, c, H->P.ncell, 0.0, 1.0);
    for (int pass = 0; pass < 4; ++pass) {
        // CG aims a little below the target so the true residual lands under it.
        PcgResult pr = pcg<T>(H, true, alpha, g, x, false, 0.5 * rtol, 0.0, default_maxit(H) - total);
        total += pr.iters;
        if (pr.status) throw Err(BLOB_RD_ENUMERIC, "non-finite value or breakdown in CG");
        true_residual(H, true, alpha, g, x, H->grid(G_T1), &rn, &gn);
        if (gn == 0.0) gn = 1.0;
        if (rn <= rtol * gn) {
            ok = true;
            break;
        }
        if (total >= default_maxit(H)) break;
        ++refinements;
    }
    launch_axpby(H->st, c, x, H->P.ncell, 0.0, 1.0);
    HIPCHK(hipStreamSynchronize(H->st));  // outputs are complete on return
    if (stt) {
        stt->outer_iters = total;
        stt->rel_resid = rn / gn;
        stt->refinements = refinements;
    }
    return ok ? BLOB_RD_OK : BLOB_RD_ENOTCONV;
}

// z = P W P r with the learned CSR (r, z device N-vectors; nv(11) scratch).
void precond_apply(blob_rd* H, const double* r, double* z) {
    // z = P W P r: the input's mean removed inside the SpMV, the output's after it
    launch_spmv_centered(H->st, H->lrn.rowptr, H->lrn.col, H->lrn.val, r, z, H->P.N);
    launch_nvec_project(H->st, z, H->P.N);
}

// y = [P] J A^+ S [P] x for N-vectors x (device) -> y (device).
template <typename T>
void schur_apply(blob_rd* H, double alpha, const double* x, double* y, double inner_rtol) {
    const Plan& P = H->P;
    hipStream_t st = H->st;
    double* xt = H->nv(2);
    launch_nvec_copy_scale(st, x, xt, P.N, 1.0, 0.0);
    if (singular(H, alpha)) launch_nvec_project(st, xt, P.N);
    // S x straight into the CG residual (zero start: r = g)
    spread_to(H, xt, 0.0, nullptr, H->grid(G_R), H->inv_h3(), nullptr);
    H->alg_bytes += (double)P.ncell * 8;
    PcgResult pr = pcg<T>(H, false, alpha, H->grid(G_R), H->grid(G_U), true, inner_rtol, 0.0, inner_maxit(H));
    if (pr.status) throw Err(BLOB_RD_ENUMERIC, "non-finite value or breakdown in inner CG");
    H->inner_iters += pr.iters;
    launch_interp(st, H->grid(G_U), P.N, P.geom, H->at<int>(P.off_base), H->at<double>(P.off_wts),
                  H->at<int>(P.off_perm), nullptr, nullptr, y, nullptr);
    if (singular(H, alpha)) launch_nvec_project(st, y, P.N);
}

// Reactive radius a0 / h of one blob, averaged over its position in the cell (Sec. IV.A),
// for the four- and three-point kernels: the diagonal 4 pi a0 D of eq. Schur_diagonal.
constexpr double kA0OverH = 1.255;
constexpr double kA0OverH3 = 0.885;

// ---- Fourier coarse level of the Schur preconditioner ----
// Integer wave vectors m with 0 < |m|^2 <= m2max, one of each pair +-m (the one whose
// first nonzero component is positive), 3 ints per vector.
std::vector<int> coarse_modes(int m2max) {
    std::vector<int> mv;
    int r = 0;
    while ((r + 1) * (r + 1) <= m2max) ++r;
    for (int mx = -r; mx <= r; ++mx)
        for (int my = -r; my <= r; ++my)
            for (int mz = -r; mz <= r; ++mz) {
                const int m2 = mx * mx + my * my + mz * mz;
                if (m2 == 0 || m2 > m2max) continue;
                const int first = mx != 0 ? mx : (my != 0 ? my : mz);
                if (first > 0) {
                    mv.push_back(mx);
                    mv.push_back(my);
                    mv.push_back(mz);
                }
            }
    return mv;
}

// Buffer layout: modes | Z, M Z, Z E^{-1}, M Z E^{-1} (K x N each) | E^{-1}, E (K x K) |
// r2, w (N) | partial dot products ((K + 1) x row chunks) | a (K). With buf == null only the
// size is computed.
size_t coarse_layout(int N, int K, char* buf, blob_rd::Coarse* C) {
    size_t o = 0;
    auto take = [&](size_t bytes) {
        size_t r = o;
        o = align_up(o + bytes);
        return buf ? buf + r : nullptr;
    };
    char* modes = take((size_t)K / 2 * 3 * 4);
    char* Z = take((size_t)K * N * 8);
    char* MZ = take((size_t)K * N * 8);
    char* ZE = take((size_t)K * N * 8);
    char* MZE = take((size_t)K * N * 8);
    char* Einv = take((size_t)K * K * 8);
    char* E = take((size_t)K * K * 8);
    char* r2 = take((size_t)N * 8);
    char* w = take((size_t)N * 8);
    char* part = take((size_t)(K + 1) * coarse_chunks(N) * 8);
    char* a = take((size_t)K * 8);
    if (C) {
        C->modes = reinterpret_cast<int*>(modes);
        C->Z = reinterpret_cast<double*>(Z);
        C->MZ = reinterpret_cast<double*>(MZ);
        C->ZE = reinterpret_cast<double*>(ZE);
        C->MZE = reinterpret_cast<double*>(MZE);
        C->Einv = reinterpret_cast<double*>(Einv);
        C->E = reinterpret_cast<double*>(E);
        C->r2 = reinterpret_cast<double*>(r2);
        C->w = reinterpret_cast<double*>(w);
        C->part = reinterpret_cast<double*>(part);
        C->a = reinterpret_cast<double*>(a);
    }
    return o;
}

// Inverse of a symmetric positive definite K x K matrix (row-major) by Cholesky;
// false if a pivot is not positive and finite.
bool spd_inverse(std::vector<double>& A, int K) {
    std::vector<double> L((size_t)K * K, 0.0);
    for (int j = 0; j < K; ++j) {
        double dj = A[(size_t)j * K + j];
        for (int k = 0; k < j; ++k) dj -= L[(size_t)j * K + k] * L[(size_t)j * K + k];
        if (!(dj > 0.0) || !std::isfinite(dj)) return false;
        const double ljj = std::sqrt(dj);
        L[(size_t)j * K + j] = ljj;
        for (int i = j + 1; i < K; ++i) {
            double v = A[(size_t)i * K + j];
            for (int k = 0; k < j; ++k) v -= L[(size_t)i * K + k] * L[(size_t)j * K + k];
            L[(size_t)i * K + j] = v / ljj;
        }
    }
    // columns of A^{-1}: L y = e_c, then L^T x = y
    std::vector<double> y(K);
    for (int c = 0; c < K; ++c) {
        for (int i = 0; i < K; ++i) {
            double v = i == c ? 1.0 : 0.0;
            for (int k = 0; k < i; ++k) v -= L[(size_t)i * K + k] * y[k];
            y[i] = v / L[(size_t)i * K + i];
        }
        for (int i = K - 1; i >= 0; --i) {
            double v = y[i];
            for (int k = i + 1; k < K; ++k) v -= L[(size_t)k * K + i] * A[(size_t)k * K + c];
            A[(size_t)i * K + c] = v / L[(size_t)i * K + i];
        }
    }
    return true;
}

// Z (cos/sin of the wave vectors at the blobs, column means removed), M Z by K Schur
// products with inner solves to inner_rtol, E = sym(Z^T M Z) and its inverse.
// Captured block-FGMRES steps read the coarse level's buffers: drop them when it changes.
void drop_fg_graphs(blob_rd* H) {
    HIPCHK(hipStreamSynchronize(H->st));
    for (auto& g : H->fg_graphs) (void)hipGraphExecDestroy(g.exec);
    H->fg_graphs.clear();
}

template <typename T>
void coarse_build(blob_rd* H, double alpha, const std::vector<int>& mv, double inner_rtol, char* buf) {
    blob_rd::Coarse& C = H->crs;
    drop_fg_graphs(H);
    C.ready = false;
    const int N = H->P.N;
    const int nm = (int)mv.size() / 3;
    const int K = 2 * nm;
    coarse_layout(N, K, buf, &C);
    hipStream_t st = H->st;
    HIPCHK(hipMemcpyAsync(C.modes, mv.data(), mv.size() * sizeof(int), hipMemcpyHostToDevice, st));
    const double two_pi = 6.283185307179586476925286766559;
    const double h = H->prm.h;
    launch_coarse_basis(st, H->at<double>(H->P.off_q), N, C.modes, nm, two_pi / (H->prm.nx * h),
                        two_pi / (H->prm.ny * h), two_pi / (H->prm.nz * h), C.Z);
    for (int j = 0; j < K; ++j) schur_apply<T>(H, alpha, C.Z + (size_t)j * N, C.MZ + (size_t)j * N, inner_rtol);
    launch_coarse_gram(st, C.Z, C.MZ, N, K, C.E);
    std::vector<double> E((size_t)K * K);
    HIPCHK(hipGetLastError());
    HIPCHK(hipMemcpyAsync(E.data(), C.E, E.size() * 8, hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    for (int i = 0; i < K; ++i)
        for (int j = 0; j < i; ++j) {
            const double v = 0.5 * (E[(size_t)i * K + j] + E[(size_t)j * K + i]);
            E[(size_t)i * K + j] = v;
            E[(size_t)j * K + i] = v;
        }
    if (!spd_inverse(E, K))
        throw Err(BLOB_RD_ENUMERIC, "coarse matrix Z^T M Z is not positive definite (too many modes for the blobs?)");
    // exactly symmetric, so the apply may read its columns as rows
    for (int i = 0; i < K; ++i)
        for (int j = 0; j < i; ++j) {
            const double v = 0.5 * (E[(size_t)i * K + j] + E[(size_t)j * K + i]);
            E[(size_t)i * K + j] = v;
            E[(size_t)j * K + i] = v;
        }
    HIPCHK(hipMemcpyAsync(C.Einv, E.data(), E.size() * 8, hipMemcpyHostToDevice, st));
    launch_coarse_rotate(st, C.Z, C.Einv, N, K, C.ZE);
    launch_coarse_rotate(st, C.MZ, C.Einv, N, K, C.MZE);
    HIPCHK(hipGetLastError());
    HIPCHK(hipStreamSynchronize(st));
    C.w0 = 4.0 * M_PI * (H->prm.kernel_w == 3 ? kA0OverH3 : kA0OverH) * h * H->prm.D;
    C.alpha = alpha;
    C.K = K;
    C.ready = true;
}

// z = B r = Q r + (I - Q M) W (I - M Q) r with Q = Z E^{-1} Z^T (M and E^{-1} symmetric, so
// E^{-1} Z^T r = (Z E^{-1})^T r and E^{-1} Z^T M w = (M Z E^{-1})^T w). W is the learned
// P W P (use_w), else the paper's diagonal 4 pi a0 D I (projected at alpha = 0): W must
// carry M^{-1}'s scale, as the coarse part does. r and z must not alias.
void coarse_apply(blob_rd* H, bool use_w, const double* r, double* z) {
    blob_rd::Coarse& C = H->crs;
    hipStream_t st = H->st;
    const int N = H->P.N, K = C.K;
    const bool sing = singular(H, C.alpha);
    launch_coarse_dots(st, C.ZE, N, K, r, C.part);                                // a = E^{-1} Z^T r
    launch_coarse_update(st, C.part, nullptr, K, -1.0, C.MZ, N, r, C.r2, C.a);    // r2 = r - M Z a
    // w = W r2 (W P: the SpMV removes the input's mean), projected only in the last pass: at
    // alpha = 0 the columns of M Z are mean-free, so w's mean changes no coefficient e
    if (use_w) launch_spmv_centered(st, H->lrn.rowptr, H->lrn.col, H->lrn.val, C.r2, C.w, N);
    else launch_nvec_copy_scale(st, C.r2, C.w, N, C.w0, 0.0);
    launch_coarse_dots(st, C.MZE, N, K, C.w, C.part, sing);                       // e = E^{-1} (M Z)^T w
    launch_coarse_update(st, C.part, C.a, K, -1.0, C.Z, N, C.w, z, nullptr, sing);  // z = P w + Z (a - e)
}

struct SaddleInfo {
    int gmres_iters = 0;
    double schur_res = 0.0;
    bool converged = false;
};

// Solve [A, S; J, 0][c; lam] = [g; phi] (phi may be null = 0) with Schur GMRES.
template <typename T>
SaddleInfo saddle_solve(blob_rd* H, double alpha, const double* g, const double* phi, double* c, double* lam,
                        double atol_schur, double final_rtol_abs, double inner_rtol, const double* lam0 = nullptr) {
    const Plan& P = H->P;
    hipStream_t st = H->st;
    const int N = P.N;
    const double h3 = H->prm.h * H->prm.h * H->prm.h;
    SaddleInfo info;
    // total source -> mean sink strength (Appendix A)
    double lbar = 0.0;
    if (alpha == 0.0) {
        unsigned np = 0;
        launch_norm_partials(st, g, P.ncell, H->part(), &np);
        launch_reduce_parts(st, H->part(), np, 2, H->dsc());
        sync_read(H, H->hbuf, H->dsc(), 16);
        lbar = h3 * H->hbuf[0] / (double)N;
        H->alg_bytes += (double)P.ncell * 8;
    }
    double* gg = H->grid(G_G);
    double* u = H->grid(G_U);
    // u0 = A^+ (g - lbar S 1); b = J u0 - phi (projected)
    double* rhs0 = H->grid(G_T2);
    spread_to(H, nullptr, -lbar, g, rhs0, H->inv_h3(), nullptr);
    H->alg_bytes += (double)P.ncell * 16;
    PcgResult pr = pcg<T>(H, false, alpha, rhs0, u, true, inner_rtol, 0.0, inner_maxit(H));
    if (pr.status) throw Err(BLOB_RD_ENUMERIC, "non-finite value in Poisson solve");
    H->inner_iters += pr.iters;
    double* b = H->nv(3);
    launch_interp(st, u, N, P.geom, H->at<int>(P.off_base), H->at<double>(P.off_wts), H->at<int>(P.off_perm), nullptr,
                  nullptr, b, nullptr);
    if (phi) launch_axpby(st, b, phi, N, 1.0, -1.0);
    if (alpha == 0.0) launch_nvec_project(st, b, N);
    // GMRES(m) with MGS on the (projected) Schur system G lt = b
    double* lt = H->nv(4);
    double* w = H->nv(5);
    // initial multiplier: zero, or lam0 - lbar (a previous time step's multipliers)
    if (lam0) {
        launch_nvec_copy_scale(st, lam0, lt, N, 1.0, -lbar);
        if (alpha == 0.0) launch_nvec_project(st, lt, N);
    } else {
        launch_nvec_copy_scale(st, nullptr, lt, N, 0.0, 0.0);
    }
    const int m = P.restart;
    double* V = H->at<double>(P.off_V);
    double* Hm = H->at<double>(P.off_H);
    const int maxit = default_maxit(H);
    bool first = lam0 == nullptr;
    bool use_w = false;
    if (H->prm.schur_precond == BLOB_RD_PRECOND_LEARNED && alpha == 0.0) {
        if (H->lrn.ready && !H->lrn.bad) use_w = true;
        else H->fallback = 1;
    }
    // right preconditioner: the coarse level built for this alpha (around W or the
    // diagonal), else W alone
    const bool coarse_on = H->crs.ready && H->crs.alpha == alpha;
    bool use_pre = use_w || coarse_on;
    auto pre = [&](const double* r, double* z) {
        if (coarse_on) coarse_apply(H, use_w, r, z);
        else precond_apply(H, r, z);
    };
    for (;;) {
        if (!first) schur_apply<T>(H, alpha, lt, w, inner_rtol);
        launch_gmres_start(st, b, w, first ? 0 : 1, V, H->at<double>(P.off_gv), N, H->gs());
        first = false;
        sync_read(H, H->hgs, H->gs(), sizeof(GmresScalars));
        info.schur_res = H->hgs->res;
        if (H->hgs->status) throw Err(BLOB_RD_ENUMERIC, "non-finite Schur residual");
        if (H->hgs->res <= atol_schur) {
            info.converged = true;
            break;
        }
        if (info.gmres_iters >= maxit) break;
        int k = 0;
        double res_prev = H->hgs->res;
        const double res_cycle0 = res_prev;
        for (; k < m && info.gmres_iters < maxit; ++k) {
            // Inexact Krylov: the matvec may be less accurate as the residual falls
            // (Bouras-Fraysse / Simoncini-Szyld relaxation); the FP64 saddle residual
            // and refinement of the caller guard the final answer.
            double tau = inner_rtol;
            if (H->relax && res_prev > 0.0) tau = std::min(1e-1, std::max(inner_rtol, atol_schur / res_prev));
            if (use_pre) {
                pre(V + (size_t)k * N, H->nv(9));
                schur_apply<T>(H, alpha, H->nv(9), V + (size_t)(k + 1) * N, tau);
            } else {
                schur_apply<T>(H, alpha, V + (size_t)k * N, V + (size_t)(k + 1) * N, tau);
            }
            launch_gmres_arnoldi(st, V, Hm, H->at<double>(P.off_cs), H->at<double>(P.off_sn),
                                 H->at<double>(P.off_gv), N, k, m, H->gs());
            ++info.gmres_iters;
            sync_read(H, H->hgs, H->gs(), sizeof(GmresScalars));
            if (H->hgs->status) throw Err(BLOB_RD_ENUMERIC, "GMRES breakdown");
            res_prev = H->hgs->res;
            if (H->hgs->res <= atol_schur || H->hgs->hk1 == 0.0) {
                ++k;
                break;
            }
        }
        if (use_pre) {
            // right preconditioning: lt += B (V y)
            launch_nvec_copy_scale(st, nullptr, H->nv(10), N, 0.0, 0.0);
            launch_gmres_update(st, V, Hm, H->at<double>(P.off_gv), H->at<double>(P.off_yv), H->nv(10), N, k, m);
            pre(H->nv(10), H->nv(9));
            launch_axpby(st, lt, H->nv(9), N, 1.0, 1.0);
            // watchdog: a full cycle that did not cut the residual 10x drops the preconditioner
            if (k == m && H->hgs->res > 0.1 * res_cycle0) {
                use_pre = false;
                H->fallback = 1;
            }
        } else {
            launch_gmres_update(st, V, Hm, H->at<double>(P.off_gv), H->at<double>(P.off_yv), lt, N, k, m);
        }
        info.schur_res = H->hgs->res;
        // The Arnoldi estimate decides; the FP64 saddle residual computed by the
        // caller checks the answer and triggers refinement if needed.
        if (H->hgs->res <= atol_schur) {
            info.converged = true;
            break;
        }
        if (info.gmres_iters >= maxit) break;
    }
    if (alpha == 0.0) launch_nvec_project(st, lt, N);
    // lam = lbar + lt ; c = A^+ (g - S lam) (+ cbar)
    launch_nvec_copy_scale(st, lt, lam, N, 1.0, lbar);
    spread_to(H, lam, 0.0, g, gg, -H->inv_h3(), nullptr);
    H->alg_bytes += (double)P.ncell * 16;
    pr = pcg<T>(H, false, alpha, gg, u, true, 0.0, final_rtol_abs, inner_maxit(H));
    if (pr.status) throw Err(BLOB_RD_ENUMERIC, "non-finite value in Poisson solve");
    H->inner_iters += pr.iters;
    launch_axpby(st, c, u, P.ncell, 0.0, 1.0);
    if (alpha == 0.0) {
        // J c + cbar = phi  ->  cbar = mean(phi - J c)
        double* jc = H->nv(6);
        launch_interp(st, c, N, P.geom, H->at<int>(P.off_base), H->at<double>(P.off_wts), H->at<int>(P.off_perm),
                      nullptr, nullptr, jc, nullptr);
        if (phi) launch_axpby(st, jc, phi, N, 1.0, -1.0);
        launch_nvec_sums(st, jc, nullptr, N, H->dsc());
        sync_read(H, H->hbuf, H->dsc(), 24);
        const double cbar = -H->hbuf[0] / (double)N;
        launch_fill(st, H->dsc() + 32, 1, cbar);
        launch_add_shift(st, c, P.ncell, H->dsc() + 32, 1.0);
        H->alg_bytes += (double)P.ncell * 16;
    }
    return info;
}

// FP64 saddle residual: t = g - A c - S lam (grid), tn = phi - J c (N); returns norms^2.
void saddle_residual(blob_rd* H, double alpha, const double* g, const double* phi, const double* c, const double* lam,
                     double* t, double* tn, double* r1sq, double* r2sq, double* gsq) {
    const Plan& P = H->P;
    const LevelDims& d = P.lev[0];
    const double s = H->prm.D / (d.h * d.h);
    double* q = H->grid(G_Q);
    launch_applyA_plain(H->st, c, q, alpha, s, d.nx, d.ny, d.nz, H->box);
    spread_to(H, lam, 0.0, q, q, H->inv_h3(), nullptr);
    unsigned np = 0;
    launch_residual_from_q(H->st, g, q, t, P.ncell, H->part(), &np);
    launch_reduce_parts(H->st, H->part(), np, 3, H->dsc());
    launch_interp(H->st, c, P.N, P.geom, H->at<int>(P.off_base), H->at<double>(P.off_wts), H->at<int>(P.off_perm),
                  nullptr, nullptr, tn, nullptr);
    if (phi)
        launch_axpby(H->st, tn, phi, P.N, -1.0, 1.0);
    else
        launch_nvec_copy_scale(H->st, tn, tn, P.N, -1.0, 0.0);
    launch_nvec_sums(H->st, tn, nullptr, P.N, H->dsc() + 3);
    sync_read(H, H->hbuf, H->dsc(), 6 * 8);
    *r1sq = H->hbuf[0];
    *gsq = H->hbuf[2];
    *r2sq = H->hbuf[4];
    H->alg_bytes += (double)P.ncell * 40;
}

template <typename T>
int absorbing_solve(blob_rd* H, double alpha, const double* f, double* c, double* lam, blob_rd_stats* stt,
                    const double* lam0 = nullptr) {
    const Plan& P = H->P;
    const double rtol = H->prm.rtol > 0.0 ? H->prm.rtol : 1e-8;
    // |f| sets the scale of the saddle residual
    unsigned np = 0;
    launch_norm_partials(H->st, f, P.ncell, H->part(), &np);
    launch_reduce_parts(H->st, H->part(), np, 2, H->dsc());
    sync_read(H, H->hbuf, H->dsc(), 16);
    double fn = std::sqrt(H->hbuf[1]);
    if (fn == 0.0) fn = 1.0;
    const double inner_rtol = std::min(1e-2, 0.05 * rtol);
    SaddleInfo si = saddle_solve<T>(H, alpha, f, nullptr, c, lam, 0.4 * rtol * fn, 0.4 * rtol * fn, inner_rtol, lam0);
    int gm = si.gmres_iters;
    double r1, r2, gsq;
    double* t = H->grid(G_T1);
    double* tn = H->nv(7);
    saddle_residual(H, alpha, f, nullptr, c, lam, t, tn, &r1, &r2, &gsq);
    double rel = std::sqrt(r1 + r2) / fn;
    int refinements = 0;
    // iterative refinement on the residual equations, in FP64 residuals
    double* dc = H->grid(G_T2);
    while (rel > rtol && refinements < 3 && gm < default_maxit(H)) {
        ++refinements;
        // correction system [A, S; J, 0][dc; dlam] = [t; tn] with t in G_T1 and tn
        // in nv(7); saddle_solve only reads them and writes dc (G_T2), dlam (nv(8)).
        double* dlam = H->nv(8);
        SaddleInfo s2 = saddle_solve<T>(H, alpha, t, tn, dc, dlam, 0.4 * rtol * fn, 0.4 * rtol * fn, inner_rtol);
        gm += s2.gmres_iters;
        launch_axpby(H->st, c, dc, P.ncell, 1.0, 1.0);
        launch_axpby(H->st, lam, dlam, P.N, 1.0, 1.0);
        saddle_residual(H, alpha, f, nullptr, c, lam, t, tn, &r1, &r2, &gsq);
        rel = std::sqrt(r1 + r2) / fn;
    }
    if (stt) {
        stt->outer_iters = gm;
        stt->rel_resid = rel;
        stt->refinements = refinements;
    }
    return rel <= rtol ? BLOB_RD_OK : BLOB_RD_ENOTCONV;
}

__global__ void k_step_rhs(const double* f, const double* c, double* g, unsigned n, double inv_dt) {
    const unsigned i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) g[i] = f[i] + inv_dt * c[i];
}

int fail(blob_rd* H, const Err& e) {
    g_last_error = e.what();
    if (H) H->err = e.what();
    return e.code;
}

template <typename F>
int guarded(blob_rd* H, blob_rd_stats* stt, F&& fn) {
    auto t0 = std::chrono::steady_clock::now();
    if (H) {
        H->vcycles = 0;
        H->alg_bytes = 0.0;
        H->inner_iters = 0;
        H->fallback = 0;
    }
    if (stt) std::memset(stt, 0, sizeof(*stt));
    int rc;
    try {
        rc = fn();
    } catch (const Err& e) {
        rc = fail(H, e);
    } catch (const std::exception& e) {
        rc = fail(H, Err(BLOB_RD_EDEVICE, e.what()));
    }
    if (stt && H) {
        stt->fallback = H->fallback;
        stt->vcycles = H->vcycles;
        stt->alg_bytes = H->alg_bytes;
        stt->inner_iters_total = H->inner_iters;
        stt->seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    }
    return rc;
}

}  // namespace

// ===========================================================================
namespace {

struct FgOpts {
    int kind = BLOB_RD_SADDLE_APPROX_SCHUR;
    int m = 5, n = 1, restart = 30, maxit = 1000;
    double rtol = 1e-8, diag = 0.0;
};

// reactive radius of a blob in units of h (Sec. IV.A): the position average of the
// four-point kernel, and the three-point kernel's value at a node

FgOpts fg_opts(const blob_rd* H, const blob_rd_saddle_opts* o) {
    FgOpts r;
    r.rtol = H->prm.rtol > 0.0 ? H->prm.rtol : 1e-8;
    if (o) {
        r.kind = o->precond;
        if (o->m > 0) r.m = o->m;
        if (o->n > 0) r.n = o->n;
        if (o->restart > 0) r.restart = o->restart;
        if (o->maxit > 0) r.maxit = o->maxit;
        if (o->rtol > 0.0) r.rtol = o->rtol;
        r.diag = o->diag;
        if (o->m < 0 || o->n < 0 || o->restart < 0 || o->maxit < 0 || !(o->rtol >= 0.0) || !(o->diag >= 0.0) ||
            !std::isfinite(o->diag) || !std::isfinite(o->rtol))
            throw Err(BLOB_RD_EINVAL, "saddle solver options must be non-negative and finite");
    }
    if (r.kind != BLOB_RD_SADDLE_DIAGONAL && r.kind != BLOB_RD_SADDLE_APPROX_SCHUR &&
        r.kind != BLOB_RD_SADDLE_LEARNED)
        throw Err(BLOB_RD_EINVAL, "unknown saddle preconditioner");
    if (r.m > H->P.restart)
        throw Err(BLOB_RD_EINVAL, "inner Krylov iterations exceed the handle's GMRES restart length");
    if (r.n > 64) throw Err(BLOB_RD_EINVAL, "at most 64 multigrid cycles per approximate solve");
    if (r.restart > kFgMaxRestart) throw Err(BLOB_RD_EINVAL, "FGMRES restart length above 1024");
    if (r.diag == 0.0) r.diag = 4.0 * M_PI * (H->prm.kernel_w == 3 ? kA0OverH3 : kA0OverH) * H->prm.h * H->prm.D;
    return r;
}


SpreadLists spread_lists(const blob_rd* H) {
    const Plan& P = H->P;
    return SpreadLists{H->ntouched, H->at<int>(P.off_tcell), H->at<int>(P.off_tptr), H->at<int>(P.off_tblob),
                       H->at<double>(P.off_tw)};
}

// q = base - A x + scale S m: the dense residual of base, then the spread term
// added at the touched cells only (M null: no spread term).
void fg_resid(blob_rd* H, double alpha, const double* base, const SpreadMult* M, double scale, const double* x,
              double* q) {
    const Plan& P = H->P;
    const LevelDims& d = P.lev[0];
    launch_residA_plain(H->st, base, x, q, alpha, H->prm.D / (d.h * d.h), d.nx, d.ny, d.nz, H->box);
    if (M) launch_spread_sparse(H->st, spread_lists(H), *M, q, q, scale, nullptr);
    H->alg_bytes += (double)P.ncell * 24;
}

// The periodic V-cycle can open from f (the opening black sweep forms the red zero-guess
// sweep as f_red / diag): level 0 in the LDS tail, or rows of the vector sweep. Not in a
// batch's V-cycle rounds, whose cycles start from a stored red sweep.
template <typename T>
bool cycle_opens_from_f(const blob_rd* H) {
    const Plan& P = H->P;
    const int t0 = std::min(H->tail_level[sizeof(T) == 4 ? 0 : 1], P.nlev - 1);
    const int vw = 16 / (int)sizeof(T);
    return !H->box && !(H->batch && H->batch_v) && (t0 == 0 || (P.lev[0].hx % vw == 0 && P.lev[0].hx >= vw));
}

void batch_run_vcycle(blob_rd* H);

// One V-cycle of the block solver: entered (r null: level-0 f and, unless from_f, the
// first red sweep already written) or from the FP64 right side r. In a batch whose
// V-cycle rounds take this handle, the executor runs the levels with the other
// members' cycles (the same kernel bodies and order, so the same results).
template <typename T>
void fg_vcycle(blob_rd* H, double alpha, const double* r, const double* cinv, bool from_f) {
    if (!(H->batch && H->batch_v)) {
        // from a right side r the entry need not store the first red sweep either
        vcycle<T>(H, alpha, r, nullptr, cinv, r == nullptr, nullptr, r ? cycle_opens_from_f<T>(H) : from_f);
        return;
    }
    const Plan& P = H->P;
    if (r) {
        const LevelDims& d = P.lev[0];
        launch_enter<T>(H->st, r, H->at<T>(P.off_lvl[0][2]), H->at<T>(P.off_lvl[0][3]), H->at<T>(P.off_lvl[0][0]),
                        d.nx, d.ny, d.nz, 1.0 / (alpha + 6.0 * H->prm.D / (d.h * d.h)), nullptr);
        H->alg_bytes += (double)P.ncell * (8 + P.esz * 1.5);
    }
    batch_run_vcycle(H);
    const int t = std::min(H->tail_level[P.esz == 4 ? 0 : 1], P.nlev - 1);
    for (int l = 0; l < t; ++l)
        H->alg_bytes += (double)P.ncell / (1 << (3 * l)) * P.esz * (kPreRestrictBytes + kProlongPostBytes);
    H->vcycles += 1;
}

// n multigrid cycles for A x = r, r = base + scale S m (M null: r = base), as a
// stationary iteration: from a zero guess the first cycle is x = V r (base
// enters the V-cycle densely and the spread term at the touched cells, so r is
// never formed), every further cycle (all of them when x holds a guess) adds
// V (r - A x).
template <typename T>
void fg_cycles(blob_rd* H, double alpha, const double* base, const SpreadMult* M, double scale, double* x,
               bool from_zero, int n, const double* cinv) {
    const Plan& P = H->P;
    const LevelDims& d = P.lev[0];
    const double inv_diag = 1.0 / (alpha + 6.0 * H->prm.D / (d.h * d.h));
    T* z0 = H->at<T>(P.off_lvl[0][0]);
    T* z1 = H->at<T>(P.off_lvl[0][1]);
    T* f0 = H->at<T>(P.off_lvl[0][2]);
    T* f1 = H->at<T>(P.off_lvl[0][3]);
    double* q = H->grid(G_Q);
    const bool from_f = from_zero && cycle_opens_from_f<T>(H);
    for (int k = 0; k < n; ++k) {
        if (k == 0 && from_zero) {
            if (H->box) {
                BoxCoef binv;
                box_coefs(H, 0, alpha, nullptr, &binv);
                launch_enter_box<T>(H->st, base, f0, f1, z0, d.nx, d.ny, d.nz, binv, nullptr);
            } else {
                launch_enter<T>(H->st, base, f0, f1, from_f ? nullptr : z0, d.nx, d.ny, d.nz, inv_diag, nullptr);
            }
            if (M)
                launch_spread_enter<T>(H->st, spread_lists(H), *M, base, scale, f0, f1, from_f ? nullptr : z0, d.nx,
                                       d.ny, inv_diag);
            H->alg_bytes += (double)P.ncell * (8 + (from_f ? 1.0 : 1.5) * P.esz);
            fg_vcycle<T>(H, alpha, nullptr, cinv, from_f);
            launch_split_to_nat<T>(H->st, z0, z1, x, d.nx, d.ny, d.nz, 0.0);
            H->alg_bytes += (double)P.ncell * (P.esz + 8);
        } else {
            fg_resid(H, alpha, base, M, scale, x, q);
            fg_vcycle<T>(H, alpha, q, cinv, false);
            launch_split_to_nat<T>(H->st, z0, z1, x, d.nx, d.ny, d.nz, 1.0);
            H->alg_bytes += (double)P.ncell * (P.esz + 16);
        }
    }
}

void fg_spread(blob_rd* H, const double* lam, const double* base_in, double* out, double scale, int add_only) {
    const Plan& P = H->P;
    spread_to(H, lam, 0.0, base_in, out, scale, nullptr);
    H->alg_bytes += (double)P.ncell * (base_in && !add_only ? 16 : 8);
}

void fg_interp(blob_rd* H, const double* c, double* out) {
    const Plan& P = H->P;
    launch_interp(H->st, c, P.N, P.geom, H->at<int>(P.off_base), H->at<double>(P.off_wts), H->at<int>(P.off_perm),
                  nullptr, nullptr, out, nullptr);
}

// [yg; yl] = [A, S; J, 0] [xg; xl]
void fg_apply_K(blob_rd* H, double alpha, const double* xg, const double* xl, double* yg, double* yl) {
    const Plan& P = H->P;
    const LevelDims& d = P.lev[0];
    launch_applyA_plain(H->st, xg, yg, alpha, H->prm.D / (d.h * d.h), d.nx, d.ny, d.nz, H->box);
    H->alg_bytes += (double)P.ncell * 16;
    fg_spread(H, xl, yg, yg, H->inv_h3(), 1);
    fg_interp(H, xg, yl);
}

// One application of the preconditioner to [vg; vf] -> [zg; zl] (steps 1-5 of
// the appendix). For A = -D L (alpha = 0): the mean multiplier from the total
// source, the blob-space mean projected out of h~, of each inner product and of
// lam~ (a constant offset of an approximate concentration only shifts J c by a
// constant, which that projection removes), and the mean concentration from the
// constraint. The right-hand sides vg - lbar S 1 and vg - S (lam~ + lbar) are
// never formed on the grid: vg enters densely and the spread terms at the
// touched cells. Grid scratch: G_Q, G_U.
template <typename T>
void fg_precond(blob_rd* H, double alpha, const FgOpts& o, const double* vg, const double* vf, double* zg,
                double* zl, bool sum_ready = false) {
    const Plan& P = H->P;
    hipStream_t st = H->st;
    const int N = P.N;
    const double h3 = H->prm.h * H->prm.h * H->prm.h;
    const double* cinv = select_cinv(H, alpha);
    const bool sing = singular(H, alpha);
    const LevelDims& d = P.lev[0];
    const SpreadLists L = spread_lists(H);
    T* z0 = H->at<T>(P.off_lvl[0][0]);
    T* z1 = H->at<T>(P.off_lvl[0][1]);
    double* ds = H->dsc() + 48;  // [0] sum of vg (already there with sum_ready), [8..10] sums of vf - J c
    double* ml = H->nv(3);       // -lbar on every blob (alpha = 0)
    // 1. concentration estimate c* from vg - lbar S 1
    if (sing) {
        if (!sum_ready) {
            unsigned np = 0;
            launch_norm_partials(st, vg, P.ncell, H->part(), &np);
            launch_reduce_parts(st, H->part(), np, 1, ds);
            H->alg_bytes += (double)P.ncell * 8;
        }
        launch_nvec_copy_scale(st, nullptr, ml, N, 0.0, 0.0);
        launch_add_shift(st, ml, N, ds, -h3 / N);
    }
    const SpreadMult m1{nullptr, ml, 1.0, 0.0};
    // With one cycle per approximate solve (periodic), c* stays in the cycle's split layout
    // and precision (its FP64 natural copy holds the same values): J c*, step 3's residual and
    // the final sum read it there, so it is never widened and narrowed again. Kept in G_Q.
    const bool split_cstar = o.n == 1 && !H->box && d.nx % 2 == 0;
    T* cs0 = reinterpret_cast<T*>(H->grid(G_Q));
    T* cs1 = cs0 + P.ncell / 2;
    const double inv_diag0 = 1.0 / (alpha + 6.0 * H->prm.D / (d.h * d.h));
    if (split_cstar) {
        const bool from_f = cycle_opens_from_f<T>(H);
        T* f0 = H->at<T>(P.off_lvl[0][2]);
        T* f1 = H->at<T>(P.off_lvl[0][3]);
        launch_enter<T>(st, vg, f0, f1, from_f ? nullptr : z0, d.nx, d.ny, d.nz, inv_diag0, nullptr);
        if (sing)
            launch_spread_enter<T>(st, L, m1, vg, H->inv_h3(), f0, f1, from_f ? nullptr : z0, d.nx, d.ny,
                                   inv_diag0);
        H->alg_bytes += (double)P.ncell * (8 + (from_f ? 1.0 : 1.5) * P.esz);
        fg_vcycle<T>(H, alpha, nullptr, cinv, from_f);
        launch_copy2<T>(st, z0, z1, cs0, cs1, P.ncell / 2);
        H->alg_bytes += (double)P.ncell * 2 * P.esz;
    } else {
        fg_cycles<T>(H, alpha, vg, sing ? &m1 : nullptr, H->inv_h3(), zg, true, o.n, cinv);
    }
    // 2. Schur-complement system for the (fluctuating) multipliers, right side J c* - vf
    double* jv = H->nv(6);
    double* hv = H->nv(4);
    if (split_cstar)
        launch_interp_split<T>(st, cs0, cs1, N, P.geom, H->at<int>(P.off_base), H->at<double>(P.off_wts),
                               H->at<int>(P.off_perm), jv);
    else
        fg_interp(H, zg, jv);
    // h~ = J c* - vf (mean removed at alpha = 0): formed on its own for the diagonal variant, by
    // the inner GMRES's start otherwise
    if (o.kind == BLOB_RD_SADDLE_DIAGONAL) {
        launch_nvec_copy_scale(st, jv, hv, N, 1.0, 0.0);
        launch_axpby(st, hv, vf, N, 1.0, -1.0);
        if (sing) launch_nvec_project(st, hv, N);
    }
    // the learned W approximates the inverse of J (-D L)^+ S on mean-zero multipliers:
    // it right-preconditions the inner GMRES (plain inner GMRES without it)
    bool learned = false;
    if (o.kind == BLOB_RD_SADDLE_LEARNED) {
        learned = sing && H->lrn.ready && !H->lrn.bad;
        if (!learned) H->fallback = 1;
    }
    if (o.kind == BLOB_RD_SADDLE_DIAGONAL) {
        launch_nvec_copy_scale(st, hv, zl, N, o.diag, 0.0);
    } else {
        // m GMRES iterations on (J A1^{-1} S [W]) y = h~ with one cycle per product, lam~ = [W] y
        double* V = H->at<double>(P.off_V);
        double* Hm = H->at<double>(P.off_H);
        double* gv = H->at<double>(P.off_gv);
        launch_gmres_start(st, jv, vf, 1, V, gv, N, H->gs(), sing ? 1 : 0);
        T* f0 = H->at<T>(P.off_lvl[0][2]);
        T* f1 = H->at<T>(P.off_lvl[0][3]);
        const size_t nh = P.ncell / 2;
        const double inv_diag = 1.0 / (alpha + 6.0 * H->prm.D / (d.h * d.h));
        const bool from_f = cycle_opens_from_f<T>(H);
        // with a Fourier coarse level built for this alpha, the inner GMRES is right-preconditioned
        // by the two-level B around W (the learned one, else the paper's diagonal for the
        // approximate-Schur variant): the long waves of the multiplier system are solved by the
        // level instead of left to the m inner iterations
        const bool use_c =
            (learned || o.kind == BLOB_RD_SADDLE_APPROX_SCHUR) && H->crs.ready && H->crs.alpha == alpha;
        for (int k = 0; k < o.m; ++k) {
            const double* vk = V + (size_t)k * N;
            if (use_c) {
                coarse_apply(H, learned, vk, H->nv(9));
                vk = H->nv(9);
            } else if (learned) {
                precond_apply(H, vk, H->nv(9));
                vk = H->nv(9);
            }
            // S v enters the V-cycle from the contribution lists: level-0 f is zero
            // outside the touched cells after the first product of the loop. With from_f
            // the opening black sweep takes the red zero-guess sweep as f_red / diag, so the
            // stale red u of the previous product need not be cleared, nor the touched red u written.
            if (!from_f) launch_zero<T>(st, z0, nh);
            if (k == 0) {
                launch_zero<T>(st, f0, nh);
                launch_zero<T>(st, f1, nh);
            }
            launch_spread_enter<T>(st, L, SpreadMult{vk, nullptr, 0.0, 0.0}, nullptr, H->inv_h3(), f0, f1,
                                   from_f ? nullptr : z0, d.nx, d.ny, inv_diag);
            H->alg_bytes += (double)nh * P.esz * ((k == 0 ? 2 : 0) + (from_f ? 0 : 1));
            fg_vcycle<T>(H, alpha, nullptr, cinv, from_f);
            launch_interp_split<T>(st, z0, z1, N, P.geom, H->at<int>(P.off_base), H->at<double>(P.off_wts),
                                   H->at<int>(P.off_perm), V + (size_t)(k + 1) * N);
            launch_gmres_arnoldi(st, V, Hm, H->at<double>(P.off_cs), H->at<double>(P.off_sn), gv, N, k, o.m,
                                 H->gs(), sing ? 1 : 0);
        }
        double* y = (learned || use_c) ? H->nv(10) : zl;
        launch_nvec_copy_scale(st, nullptr, y, N, 0.0, 0.0);
        launch_gmres_update(st, V, Hm, gv, H->at<double>(P.off_yv), y, N, o.m, o.m);
        if (use_c) coarse_apply(H, learned, y, zl);
        else if (learned) precond_apply(H, y, zl);
        H->inner_iters += o.m;
    }
    if (sing) launch_nvec_project(st, zl, N);
    // 3. corrected concentration: cycles on A c = vg - S (lam~ + lbar), started at c*
    const SpreadMult m2{zl, sing ? ml : nullptr, -1.0, 0.0};
    if (sing && o.n == 1) {
        // one cycle; 4. the mean concentration from J c* + J z before z is added,
        // so the shift rides on the pass that adds z
        if (split_cstar) {
            // the entry of vg - A c* - S (lam~ + lbar) straight from the split c*
            const bool from_f = cycle_opens_from_f<T>(H);
            T* f0 = H->at<T>(P.off_lvl[0][2]);
            T* f1 = H->at<T>(P.off_lvl[0][3]);
            const double s0 = H->prm.D / (d.h * d.h);
            launch_resid_enter<T>(st, vg, cs0, cs1, f0, f1, from_f ? nullptr : z0, d.nx, d.ny, d.nz, alpha, s0,
                                  inv_diag0);
            launch_resid_spread_enter<T>(st, L, m2, vg, cs0, cs1, -H->inv_h3(), f0, f1, from_f ? nullptr : z0, d.nx,
                                         d.ny, d.nz, alpha, s0, inv_diag0);
            H->alg_bytes += (double)P.ncell * (8 + P.esz * (from_f ? 2.0 : 2.5));
            fg_vcycle<T>(H, alpha, nullptr, cinv, from_f);
        } else {
            double* q = H->grid(G_Q);
            fg_resid(H, alpha, vg, &m2, -H->inv_h3(), zg, q);
            fg_vcycle<T>(H, alpha, q, cinv, false);
        }
        double* jz = H->nv(5);
        launch_interp_split<T>(st, z0, z1, N, P.geom, H->at<int>(P.off_base), H->at<double>(P.off_wts),
                               H->at<int>(P.off_perm), jz);
        launch_axpby(st, jz, vf, N, -1.0, 1.0);  // vf - J z
        launch_axpby(st, jz, jv, N, 1.0, -1.0);  // vf - J z - J c*
        launch_nvec_sums(st, jz, nullptr, N, ds + 8);
        if (split_cstar) {
            launch_split_add_to_nat<T>(st, cs0, cs1, z0, z1, zg, d.nx, d.ny, d.nz, ds + 8, 1.0 / N);
            H->alg_bytes += (double)P.ncell * (2 * P.esz + 8);
        } else {
            launch_split_to_nat<T>(st, z0, z1, zg, d.nx, d.ny, d.nz, 1.0, ds + 8, 1.0 / N);
            H->alg_bytes += (double)P.ncell * (P.esz + 16);
        }
    } else if (split_cstar) {
        // one cycle from c*: the entry of vg - A c* - S lam~ straight from the split c*
        const bool from_f = cycle_opens_from_f<T>(H);
        T* f0 = H->at<T>(P.off_lvl[0][2]);
        T* f1 = H->at<T>(P.off_lvl[0][3]);
        const double s0 = H->prm.D / (d.h * d.h);
        launch_resid_enter<T>(st, vg, cs0, cs1, f0, f1, from_f ? nullptr : z0, d.nx, d.ny, d.nz, alpha, s0, inv_diag0);
        launch_resid_spread_enter<T>(st, L, m2, vg, cs0, cs1, -H->inv_h3(), f0, f1, from_f ? nullptr : z0, d.nx, d.ny,
                                     d.nz, alpha, s0, inv_diag0);
        fg_vcycle<T>(H, alpha, nullptr, cinv, from_f);
        launch_split_add_to_nat<T>(st, cs0, cs1, z0, z1, zg, d.nx, d.ny, d.nz, nullptr, 0.0);
        H->alg_bytes += (double)P.ncell * (16 + P.esz * (from_f ? 4.0 : 4.5));
    } else {
        fg_cycles<T>(H, alpha, vg, &m2, -H->inv_h3(), zg, false, o.n, cinv);
        if (sing) {
            // 4. mean concentration: mean over blobs of vf - J c
            fg_interp(H, zg, jv);
            launch_axpby(st, jv, vf, N, -1.0, 1.0);
            launch_nvec_sums(st, jv, nullptr, N, ds + 8);
            launch_add_shift(st, zg, P.ncell, ds + 8, 1.0 / N);
            H->alg_bytes += (double)P.ncell * 16;
        }
    }
    // 5. lam = lam~ + lbar
    if (sing) launch_add_shift(st, zl, N, ds, h3 / N);
}

// Flexible GMRES (right preconditioned, restarted, modified Gram-Schmidt) on
// [A, S; J, 0][c; lam] = [f; phi] from a zero guess (warm: from (c, lam)), with
// phi = -cb on every blob in a box held at cb (the lifted system) and 0 otherwise.
// Every cycle starts from the true FP64 residual b - K x, which also decides
// convergence at the end.
template <typename T>
int fg_solve(blob_rd* H, double alpha, const FgOpts& o, const double* f, double* c, double* lam, char* ws,
             blob_rd_stats* stt, bool warm = false) {
    const Plan& P = H->P;
    hipStream_t st = H->st;
    const size_t ncell = P.ncell, n = ncell + (size_t)P.N, stride = fg_stride(P);
    const int m = o.restart, ld = m + 1;
    double* V = reinterpret_cast<double*>(ws);
    double* Z = V + (size_t)(m + 1) * stride;
    double* Hd = Z + (size_t)m * stride;
    double* cs = Hd + (size_t)ld * m;
    double* sn = cs + ld;
    double* gv = sn + ld;
    double* yv = gv + ld;
    double* sd = yv + ld;  // [0] beta, [2..3] Givens outputs, [4..5] norms of a warm start, [6] |w|^2, [7] redo flag
    double* c2 = sd + 8;   // dots of the re-orthogonalisation pass
    int* redo = reinterpret_cast<int*>(sd + 7);
    // classical Gram-Schmidt in groups of up to 8 basis vectors per pass over w, as far as the
    // partial-sum buffer allows (modified Gram-Schmidt otherwise)
    const unsigned cgs_nb = fg_cgs_blocks(n);
    const int group = (int)std::min<long long>(8, (long long)(3 * P.part_cap / cgs_nb) - 1);
    // re-orthogonalise when the projection removed all but this fraction of |w| (always, with
    // the handle's reorth_always)
    const double kReorth = H->reorth_always ? 1e150 : 0.1;
    double bnorm = -1.0, rel = 0.0, prev_rel = 0.0;
    const double phi = H->box ? -H->cb : 0.0;
    // normalising a basis vector also sums its grid part for the preconditioner's mean step
    // (singular A) when the partial-sum buffer holds one partial per block
    const bool fuse_sum = singular(H, alpha) && red_blocks(n) <= 3 * P.part_cap;
    auto scale_basis = [&](hipStream_t s, double* v, const double* hv) {
        if (fuse_sum) {
            unsigned nps = 0;
            launch_fg_scale_sum(s, v, hv, n, ncell, H->part(), &nps);
            launch_reduce_parts(s, H->part(), nps, 1, H->dsc() + 48);
        } else {
            launch_fg_scale(s, v, hv, n);
        }
    };
    // the Arnoldi steps run as captured graphs (not in a batch's V-cycle rounds, which
    // rendezvous with the executor on the host, nor where the call must not allocate)
    const bool graphs = H->use_graphs && H->fg_capture && !H->batch;
    const bool ahead = H->fg_capture && !H->batch && H->fg_ahead > 0;  // steps issued ahead of the host's reads
    if (ahead)
        for (auto& e : H->fg_ev)
            if (!e) HIPCHK(hipEventCreateWithFlags(&e, hipEventDisableTiming));
    (void)select_cinv(H, alpha);  // its upload, if any, happens outside any capture
    if (warm) {
        // (c, lam) hold the initial guess; the scale of the residual is |b| = |[f; phi]|
        unsigned np = 0;
        launch_norm_partials(st, f, ncell, H->part(), &np);
        launch_reduce_parts(st, H->part(), np, 2, sd + 4);
        sync_read(H, H->hbuf, sd + 4, 16);
        const double bb = H->hbuf[1] + (double)P.N * phi * phi;
        bnorm = bb > 0.0 ? std::sqrt(bb) : 1.0;
        H->alg_bytes += (double)ncell * 8;
    } else {
        launch_fill(st, c, ncell, 0.0);
        launch_fill(st, lam, P.N, 0.0);
    }
    int its = 0, cycles = 0, stalled = 0;
    bool sub = warm;
    for (;;) {
        if (sub) fg_apply_K(H, alpha, c, lam, V, V + ncell);
        unsigned np = 0;
        launch_fg_resid(st, V, f, ncell, n, sub ? 1 : 0, H->part(), &np, phi);
        launch_fg_fin(st, H->part(), np, sd, 1);
        H->alg_bytes += (double)n * (sub ? 24 : 16);
        sync_read(H, H->hbuf, sd, 8);
        const double beta = H->hbuf[0];
        if (!std::isfinite(beta)) throw Err(BLOB_RD_ENUMERIC, "non-finite FGMRES residual");
        if (bnorm < 0.0) bnorm = beta > 0.0 ? beta : 1.0;  // zero start: the first residual is b
        rel = beta / bnorm;
        if (rel <= o.rtol || its >= o.maxit) break;
        // A restarted cycle cannot raise the true residual; two cycles in a row that cut it
        // by less than 1 % mean the rounding floor of the residual is above rtol.
        stalled = (cycles > 0 && rel > 0.99 * prev_rel) ? stalled + 1 : 0;
        if (stalled >= 2) break;
        prev_rel = rel;
        ++cycles;
        scale_basis(st, V, sd);
        launch_fg_gstart(st, gv, ld, sd);
        H->alg_bytes += (double)n * 16;
        int k = 0;
        // issue Arnoldi step j: its kernels (or its captured graph), then the copy of its
        // residual estimate and sub-diagonal to hbuf[8 + 2 (j & 1)], recorded by fg_ev[j & 1]
        auto issue = [&](int j) {
            // one Arnoldi step: z_j = M^-1 v_j, w = K z_j orthogonalised against the basis and
            // normalised, the Givens rotation of column j (all on the handle's current stream)
            auto step = [&]() {
                hipStream_t s = H->st;
                double* vj = V + (size_t)j * stride;
                double* zj = Z + (size_t)j * stride;
                double* w = V + (size_t)(j + 1) * stride;
                fg_precond<T>(H, alpha, o, vj, vj + ncell, zj, zj + ncell, fuse_sum);
                fg_apply_K(H, alpha, zj, zj + ncell, w, w + ncell);
                double* col = Hd + (size_t)j * ld;
                if (group >= 1) {
                    // h = V^T w, w -= V h, |w|; once more (dots into c2, h += c2) when |w| fell below
                    // kReorth of its length before the projection
                    const int mv = j + 1;
                    launch_fg_cgs_dots(s, w, V, stride, n, mv, group, col, sd + 6, H->part(), nullptr);
                    launch_fg_cgs_update(s, w, V, stride, n, col, mv, H->part(), nullptr, col + j + 1, sd + 6,
                                         kReorth * kReorth, redo, nullptr, nullptr);
                    launch_fg_cgs_dots(s, w, V, stride, n, mv, group, c2, nullptr, H->part(), redo);
                    launch_fg_cgs_update(s, w, V, stride, n, c2, mv, H->part(), redo, col + j + 1, nullptr, 0.0,
                                         nullptr, col, c2);
                    const int passes = (mv + group - 1) / group;
                    H->alg_bytes += (double)n * 8 * ((double)mv + passes + (mv + 2));
                } else {
                    unsigned np2 = 0;
                    for (int i = 0; i <= j + 1; ++i) {
                        const double* vprev = i > 0 ? V + (size_t)(i - 1) * stride : nullptr;
                        const double* vnext = i <= j ? V + (size_t)i * stride : nullptr;
                        launch_fg_mgs(s, w, vprev, i > 0 ? col + (i - 1) : nullptr, vnext, n, H->part(), &np2);
                        launch_fg_fin(s, H->part(), np2, col + i, i == j + 1);
                        H->alg_bytes += (double)n * 8 * ((vprev ? 3 : 1) + (vnext ? 1 : 0));
                    }
                }
                scale_basis(s, w, col + j + 1);
                H->alg_bytes += (double)n * 16;
                launch_fg_givens(s, Hd, ld, cs, sn, gv, j, sd + 2);
            };
            if (graphs) {
                // replay the captured step of this j (capture it on first use)
                const bool learned = o.kind == BLOB_RD_SADDLE_LEARNED && singular(H, alpha) && H->lrn.ready &&
                                     !H->lrn.bad;
                blob_rd::FgGraph* ge = nullptr;
                for (auto& g : H->fg_graphs)
                    if (g.ws == ws && g.j == j && g.esz == (int)sizeof(T) && g.kind == o.kind && g.m == o.m &&
                        g.n == o.n && g.restart == m && g.group == group && g.alpha == alpha && g.fuse == fuse_sum &&
                        g.learned == learned)
                        ge = &g;
                if (!ge) {
                    if (!H->cap_stream) HIPCHK(hipStreamCreateWithFlags(&H->cap_stream, hipStreamNonBlocking));
                    const double b0 = H->alg_bytes;
                    const int v0 = H->vcycles, i0 = H->inner_iters, f0 = H->fallback;
                    hipStream_t keep = H->st;
                    H->st = H->cap_stream;
                    HIPCHK(hipStreamBeginCapture(H->cap_stream, hipStreamCaptureModeThreadLocal));
                    step();
                    hipGraph_t graph;
                    H->st = keep;
                    HIPCHK(hipStreamEndCapture(H->cap_stream, &graph));
                    hipGraphExec_t exec;
                    const hipError_t e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
                    (void)hipGraphDestroy(graph);
                    HIPCHK(e);
                    H->fg_graphs.push_back({ws, j, (int)sizeof(T), o.kind, o.m, o.n, m, group, alpha, fuse_sum,
                                            learned, exec, H->alg_bytes - b0, H->vcycles - v0, H->inner_iters - i0,
                                            H->fallback});
                    ge = &H->fg_graphs.back();
                    H->alg_bytes = b0;
                    H->vcycles = v0;
                    H->inner_iters = i0;
                    H->fallback = f0;
                }
                HIPCHK(hipGraphLaunch(ge->exec, st));
                H->alg_bytes += ge->bytes;
                H->vcycles += ge->vcycles;
                H->inner_iters += ge->inner;
                H->fallback = std::max(H->fallback, ge->fallback);
            } else {
                step();
            }
            if (ahead) {
                HIPCHK(hipMemcpyAsync(H->hbuf + 8 + 2 * (j & 1), sd + 2, 16, hipMemcpyDeviceToHost, st));
                HIPCHK(hipEventRecord(H->fg_ev[j & 1], st));
            }
        };
        // Step j + 1 goes onto the stream before the host reads step j's estimate when the
        // estimates so far (the last contraction, with a margin of 10) say step j will not reach
        // the tolerance: the read and the next launch then overlap step j instead of leaving
        // the GPU idle. A step writes only column j of H, Z_j, V_{j+1} and the Givens entries
        // j, j + 1, so a step issued past convergence changes nothing the update below reads;
        // it is not counted. (Not in a batch, whose V-cycle rounds meet the executor on the
        // host, nor where the call must not allocate: there every step is read before the next.)
        double e1 = beta, e2 = -1.0;  // estimates after the last two steps read (beta before the first)
        for (int j = 0; j < m && its < o.maxit; ++j) {
            if (j == 0 || !ahead) issue(j);
            bool spec = false;
            double b0 = 0.0;
            int v0 = 0, i0 = 0;
            if (ahead && j + 1 < m && its + 1 < o.maxit) {
                const double q = e2 > 0.0 ? std::min(1.0, e1 / e2) : 1.0;
                if (H->fg_ahead == 2 || e1 * q > 10.0 * o.rtol * bnorm) {
                    b0 = H->alg_bytes;
                    v0 = H->vcycles;
                    i0 = H->inner_iters;
                    issue(j + 1);
                    spec = true;
                }
            }
            double res, sub_diag;
            if (ahead) {
                HIPCHK(hipEventSynchronize(H->fg_ev[j & 1]));
                res = H->hbuf[8 + 2 * (j & 1)];
                sub_diag = H->hbuf[9 + 2 * (j & 1)];
            } else {
                sync_read(H, H->hbuf, sd + 2, 16);
                res = H->hbuf[0];
                sub_diag = H->hbuf[1];
            }
            ++its;
            k = j + 1;
            if (!std::isfinite(res) || !std::isfinite(sub_diag)) throw Err(BLOB_RD_ENUMERIC, "FGMRES breakdown");
            if (res <= o.rtol * bnorm || sub_diag == 0.0) {
                if (spec) {
                    H->alg_bytes = b0;
                    H->vcycles = v0;
                    H->inner_iters = i0;
                }
                break;
            }
            e2 = e1;
            e1 = res;
            if (ahead && !spec && j + 1 < m && its < o.maxit) issue(j + 1);
        }
        launch_fg_backsolve(st, Hd, ld, gv, yv, k);
        launch_fg_update(st, c, Z, stride, 0, ncell, k, yv);
        launch_fg_update(st, lam, Z, stride, ncell, P.N, k, yv);
        H->alg_bytes += (double)n * 8 * (k + 2);
        sub = true;
    }
    if (stt) {
        stt->outer_iters = its;
        stt->rel_resid = rel;
        stt->refinements = cycles > 0 ? cycles - 1 : 0;
    }
    return rel <= o.rtol ? BLOB_RD_OK : BLOB_RD_ENOTCONV;
}


// Block solver options of a handle created with saddle_solver != BLOB_RD_SOLVER_SCHUR
// (the learned inner preconditioning only where W applies, alpha = 0).
FgOpts handle_fg_opts(const blob_rd* H, double alpha) {
    blob_rd_saddle_opts o{};
    o.precond = (H->prm.saddle_solver == BLOB_RD_SOLVER_BLOCK_LEARNED && singular(H, alpha))
                    ? BLOB_RD_SADDLE_LEARNED
                    : BLOB_RD_SADDLE_APPROX_SCHUR;
    o.restart = H->P.restart;
    o.maxit = H->prm.max_iter;
    return fg_opts(H, &o);
}

// A box held at cb on its faces: the solves work on u = c - cb (the ghost 2 cb - c
// becomes -u), and a blob whose kernel support lies inside the box has J 1 = 1, so
// (alpha I - D L_cb + S kappa J) c = f becomes (alpha I - D L_0 + S kappa J) u =
// f - alpha cb - cb S kappa, and the saddle point's constraint J c = 0 becomes J u = -cb.
// box_lift writes out = f - alpha cb [- cb S kappa] (out may alias f).
void box_lift(blob_rd* H, double alpha, const double* f, double* out, bool kappa_term) {
    const Plan& P = H->P;
    launch_nvec_copy_scale(H->st, f, out, (int)P.ncell, 1.0, -alpha * H->cb);
    if (kappa_term && P.N > 0 && H->has_kappa)
        spread_to(H, H->at<double>(P.off_kappa), 0.0, out, out, -H->cb * H->inv_h3(), nullptr);
    H->alg_bytes += (double)P.ncell * 16;
}

// v += a on a grid vector
void grid_shift(blob_rd* H, double* v, double a) {
    launch_nvec_copy_scale(H->st, v, v, (int)H->P.ncell, 1.0, a);
    H->alg_bytes += (double)H->P.ncell * 16;
}

// block FGMRES of the handle's options on the saddle point with right side f
// (lifted in a box); c and lam hold the guess when warm.
template <typename T>
int fg_entry(blob_rd* H, double alpha, const FgOpts& o, const double* f, double* c, double* lam, char* ws,
             blob_rd_stats* stt, bool warm) {
    if (!H->box) return fg_solve<T>(H, alpha, o, f, c, lam, ws, stt, warm);
    double* g = H->grid(G_G);
    box_lift(H, alpha, f, g, false);
    if (warm) grid_shift(H, c, -H->cb);
    const int rc = fg_solve<T>(H, alpha, o, g, c, lam, ws, stt, warm);
    grid_shift(H, c, H->cb);
    HIPCHK(hipStreamSynchronize(H->st));
    return rc;
}

// multigrid CG on the reactive system with right side f (lifted in a box); c holds the guess
template <typename T>
int reactive_entry(blob_rd* H, double alpha, const double* f, double* c, blob_rd_stats* stt) {
    if (!H->box) return reactive_solve<T>(H, alpha, f, c, stt);
    double* g = H->grid(G_G);
    box_lift(H, alpha, f, g, true);
    grid_shift(H, c, -H->cb);
    const int rc = reactive_solve<T>(H, alpha, g, c, stt);
    grid_shift(H, c, H->cb);
    HIPCHK(hipStreamSynchronize(H->st));
    return rc;
}

}  // namespace

// ===========================================================================
// C ABI
// ===========================================================================
extern "C" {

size_t blob_rd_workspace_bytes(const blob_rd_params* p) {
    Plan P;
    std::string why;
    if (make_plan(p, &P, &why) != 0) {
        g_last_error = why;
        return 0;
    }
    return P.total;
}

}  // extern "C"

namespace {
void own_build(blob_rd* H);
}

extern "C" {

int blob_rd_create(const blob_rd_params* p, blob_rd_t* out) {
    if (!out) {
        g_last_error = "null output handle";
        return BLOB_RD_EINVAL;
    }
    *out = nullptr;
    blob_rd* H = new blob_rd();
    std::string why;
    int rc = make_plan(p, &H->P, &why);
    if (rc != 0) {
        g_last_error = why;
        delete H;
        return rc;
    }
    if (!p->workspace || p->workspace_bytes < H->P.total) {
        g_last_error = "workspace missing or smaller than blob_rd_workspace_bytes()";
        delete H;
        return BLOB_RD_ENOMEM;
    }
    H->prm = *p;
    H->st = (hipStream_t)p->stream;
    H->box = p->boundary == BLOB_RD_BOUNDARY_DIRICHLET;
    H->cb = H->box ? p->boundary_value : 0.0;
    if (const char* g = std::getenv("BLOB_RD_GRAPHS")) H->use_graphs = std::atoi(g) != 0;
    for (auto& row : H->bs)
        for (int& v : row) v = kBlock;
    if (const char* g = std::getenv("BLOB_RD_RELAX")) H->relax = std::atoi(g) != 0;
    if (const char* g = std::getenv("BLOB_RD_BLOCKED")) H->blocked = std::atoi(g) != 0;
    if (const char* g = std::getenv("BLOB_RD_FG_REORTH")) H->reorth_always = std::atoi(g) != 0;
    if (const char* g = std::getenv("BLOB_RD_FG_AHEAD")) H->fg_ahead = std::min(2, std::max(0, std::atoi(g)));
    // Align the workspace base to 256 bytes.
    uintptr_t base = (uintptr_t)p->workspace;
    H->ws = (char*)((base + 255) & ~(uintptr_t)255);
    try {
        HIPCHK(hipHostMalloc((void**)&H->hsc, sizeof(Scalars), hipHostMallocDefault));
        HIPCHK(hipHostMalloc((void**)&H->hgs, sizeof(GmresScalars), hipHostMallocDefault));
        HIPCHK(hipHostMalloc((void**)&H->hbuf, 64 * sizeof(double), hipHostMallocDefault));
        const Plan& P = H->P;
        const int N = P.N;
        hipStream_t st = H->st;
        HIPCHK(hipMemsetAsync(H->at<int>(P.off_counts), 0, (size_t)P.ntiles * 4, st));
        HIPCHK(hipMemsetAsync(H->at<int>(P.off_cursor), 0, (size_t)P.ntiles * 4, st));
        HIPCHK(hipMemsetAsync(H->grid(G_Q), 0, P.ncell * 8, st));
        HIPCHK(hipMemsetAsync(H->grid(G_P), 0, P.ncell * 8, st));
        HIPCHK(hipMemsetAsync(H->grid(G_P2), 0, P.ncell * 8, st));
        if (N > 0) {
            // Validate inputs on the host before any kernel derives indices from them.
            std::vector<double> hq((size_t)N * 3), hk;
            HIPCHK(hipMemcpyAsync(hq.data(), p->q, (size_t)N * 24, hipMemcpyDeviceToHost, st));
            if (p->kappa) {
                hk.resize(N);
                HIPCHK(hipMemcpyAsync(hk.data(), p->kappa, (size_t)N * 8, hipMemcpyDeviceToHost, st));
            }
            HIPCHK(hipStreamSynchronize(st));
            for (double v : hq)
                if (!std::isfinite(v) || std::fabs(v) > 1e12) throw Err(BLOB_RD_EINVAL, "q contains non-finite or huge values");
            if (H->box) {
                // the kernel support of every blob stays off the boundary cells
                const double edge[3] = {p->nx * p->h, p->ny * p->h, p->nz * p->h};
                for (int i = 0; i < N; ++i)
                    for (int a = 0; a < 3; ++a) {
                        const double v = hq[(size_t)i * 3 + a];
                        if (v < 3.0 * p->h || v > edge[a] - 3.0 * p->h)
                            throw Err(BLOB_RD_EINVAL,
                                      "in a Dirichlet box every blob must lie at least 3h inside each face");
                    }
            }
            for (double v : hk)
                if (!std::isfinite(v) || v < 0.0) throw Err(BLOB_RD_EINVAL, "kappa must be finite and >= 0");
            HIPCHK(hipMemcpyAsync(H->at<double>(P.off_q), p->q, (size_t)N * 24, hipMemcpyDeviceToDevice, st));
            if (p->kappa)
                HIPCHK(hipMemcpyAsync(H->at<double>(P.off_kappa), p->kappa, (size_t)N * 8, hipMemcpyDeviceToDevice,
                                      st));
            else
                HIPCHK(hipMemsetAsync(H->at<double>(P.off_kappa), 0, (size_t)N * 8, st));
            launch_blob_setup(st, H->at<double>(P.off_q), N, P.geom, H->at<int>(P.off_base),
                              H->at<double>(P.off_wts), H->at<int>(P.off_tile), H->at<int>(P.off_counts));
        }
        launch_bin_scan(st, H->at<int>(P.off_counts), P.ntiles, H->at<int>(P.off_offsets));
        if (N > 0) {
            launch_bin_scatter(st, H->at<int>(P.off_tile), N, H->at<int>(P.off_offsets), H->at<int>(P.off_cursor),
                               H->at<int>(P.off_perm));
            launch_bin_sort(st, H->at<int>(P.off_offsets), P.ntiles, H->at<int>(P.off_perm));
            // contribution lists of the spread: count per tile, scan, fill
            int* cnt = H->at<int>(P.off_sp_cnt);
            int* offE = H->at<int>(P.off_sp_off);
            int* offC = offE + P.ntiles + 1;
            launch_spread_plan(st, 0, P.geom, H->at<int>(P.off_base), H->at<double>(P.off_wts),
                               H->at<int>(P.off_offsets), H->at<int>(P.off_perm), cnt, nullptr, nullptr, nullptr,
                               nullptr, nullptr, nullptr);
            launch_bin_scan(st, cnt, P.ntiles, offE);
            launch_bin_scan(st, cnt + P.ntiles, P.ntiles, offC);
            launch_spread_plan(st, 1, P.geom, H->at<int>(P.off_base), H->at<double>(P.off_wts),
                               H->at<int>(P.off_offsets), H->at<int>(P.off_perm), nullptr, offE, offC,
                               H->at<int>(P.off_tcell), H->at<int>(P.off_tptr), H->at<int>(P.off_tblob),
                               H->at<double>(P.off_tw));
            int nt[2] = {0, 0};
            HIPCHK(hipMemcpyAsync(&nt[0], offE + P.ntiles, 4, hipMemcpyDeviceToHost, st));
            HIPCHK(hipMemcpyAsync(&nt[1], offC + P.ntiles, 4, hipMemcpyDeviceToHost, st));
            HIPCHK(hipStreamSynchronize(st));
            if (nt[0] < 0 || nt[0] > 64 * N || nt[1] < 0 || nt[1] > nt[0])
                throw Err(BLOB_RD_EDEVICE, "spread contribution lists out of range");
            H->ntouched = nt[1];
            launch_nvec_sums(st, H->at<double>(P.off_kappa), nullptr, N, H->dsc());
            sync_read(H, H->hbuf, H->dsc(), 24);
            H->sum_kappa = H->hbuf[0];
            H->has_kappa = p->kappa != nullptr;
            if (!std::isfinite(H->sum_kappa)) throw Err(BLOB_RD_EINVAL, "kappa contains non-finite values");
        }
        HIPCHK(hipGetLastError());
        HIPCHK(hipStreamSynchronize(st));
        select_cinv(H, 0.0);
        // LDS budget of the coarse tail: the device limit per block, capped at 160 KiB.
        int dev = 0, lds = 0;
        HIPCHK(hipGetDevice(&dev));
        HIPCHK(hipDeviceGetAttribute(&lds, hipDeviceAttributeMaxSharedMemoryPerBlock, dev));
        const size_t budget = std::min<size_t>((size_t)lds, 160 * 1024);
        H->tail_level[0] = tail_start(P, 4, budget);
        H->tail_level[1] = tail_start(P, 8, budget);
        const int Lc = P.nlev - 1;
        if (H->tail_level[0] < Lc) {
            const size_t need = make_tail<float>(H, H->tail_level[0], 0.0).lds_bytes;
            if (need > 48 * 1024) HIPCHK(H->box ? tail_box_set_lds<float>(need) : tail_set_lds<float>(need));
        }
        if (H->tail_level[1] < Lc) {
            const size_t need = make_tail<double>(H, H->tail_level[1], 0.0).lds_bytes;
            if (need > 48 * 1024) HIPCHK(H->box ? tail_box_set_lds<double>(need) : tail_set_lds<double>(need));
        }
        if (H->blocked) {
            HIPCHK(blocked_set_lds<float>());
            HIPCHK(blocked_set_lds<double>());
        }
        H->noalloc = &scratch_slot();
        if (P.off_net) {
            // the handle's own network starts untrained: W is then the diagonal of eq. Schur_diagonal
            if (blob_rd_net_create(H->ws + P.off_net, net_bytes(), (void*)st, &H->own_net) != BLOB_RD_OK)
                throw Err(BLOB_RD_EDEVICE, "network set-up failed: " + g_last_error);
            HIPCHK(hipStreamSynchronize(st));
            own_build(H);
        }
    } catch (const Err& e) {
        g_last_error = e.what();
        blob_rd_destroy(H);
        return e.code;
    }
    *out = H;
    return BLOB_RD_OK;
}

int blob_rd_destroy(blob_rd_t H) {
    if (!H) return BLOB_RD_OK;
    if (H->batch_ev) (void)hipEventDestroy(H->batch_ev);
    for (auto& e : H->fg_ev)
        if (e) (void)hipEventDestroy(e);
    for (auto& g : H->fg_graphs) (void)hipGraphExecDestroy(g.exec);
    H->fg_graphs.clear();
    if (H->own_net) blob_rd_net_destroy(H->own_net);
    for (auto& g : H->graphs) (void)hipGraphExecDestroy(g.exec);
    H->graphs.clear();
    if (H->cap_stream) (void)hipStreamDestroy(H->cap_stream);
    if (H->hsc) (void)hipHostFree(H->hsc);
    if (H->hgs) (void)hipHostFree(H->hgs);
    if (H->hbuf) (void)hipHostFree(H->hbuf);
    delete H;
    return BLOB_RD_OK;
}

const char* blob_rd_last_error(blob_rd_t H) {
    (void)H;
    return g_last_error.c_str();
}

int blob_rd_solve_reactive(blob_rd_t H, double alpha, const double* f, double* c, blob_rd_stats* stt) {
    if (!H || !f || !c) return g_last_error = "null argument", BLOB_RD_EINVAL;
    if (!(alpha >= 0.0) || !std::isfinite(alpha)) return g_last_error = "alpha must be >= 0", BLOB_RD_EINVAL;
    if (alpha == 0.0 && !(H->sum_kappa > 0.0) && !H->box)
        return g_last_error = "steady reactive system with zero total rate is singular", BLOB_RD_ESINGULAR;
    return guarded(H, stt, [&]() {
        int rc = H->P.esz == 4 ? reactive_entry<float>(H, alpha, f, c, stt) : reactive_entry<double>(H, alpha, f, c, stt);
        HIPCHK(hipGetLastError());
        return rc;
    });
}

int blob_rd_step(blob_rd_t H, double dt, const double* f, double* c, blob_rd_stats* stt) {
    if (!H || !f || !c) return g_last_error = "null argument", BLOB_RD_EINVAL;
    if (!(dt > 0.0) || !std::isfinite(dt)) return g_last_error = "dt must be positive", BLOB_RD_EINVAL;
    return guarded(H, stt, [&]() {
        double* g = H->grid(G_G);
        hipLaunchKernelGGL(k_step_rhs, dim3(nblocks(H->P.ncell)), dim3(kBlock), 0, H->st, f, c, g,
                           (unsigned)H->P.ncell, 1.0 / dt);
        H->alg_bytes += (double)H->P.ncell * 24;
        int rc = H->P.esz == 4 ? reactive_entry<float>(H, 1.0 / dt, g, c, stt)
                               : reactive_entry<double>(H, 1.0 / dt, g, c, stt);
        HIPCHK(hipGetLastError());
        return rc;
    });
}

int blob_rd_step_absorbing(blob_rd_t H, double dt, const double* f, double* c, double* lambda, int warm,
                           blob_rd_stats* stt) {
    if (!H || !f || !c || !lambda) return g_last_error = "null argument", BLOB_RD_EINVAL;
    if (H->P.N <= 0) return g_last_error = "absorbing step needs at least one blob", BLOB_RD_EINVAL;
    if (!(dt > 0.0) || !std::isfinite(dt)) return g_last_error = "dt must be positive", BLOB_RD_EINVAL;
    if (H->box && H->prm.saddle_solver == BLOB_RD_SOLVER_SCHUR)
        return g_last_error = "absorbing solves in a Dirichlet box need saddle_solver BLOCK", BLOB_RD_EINVAL;
    return guarded(H, stt, [&]() {
        // g = c^n/dt + f in its own buffer: c is overwritten by c^{n+1}, and the
        // saddle residual and refinement read g after that
        double* g = H->grid(G_S);
        hipLaunchKernelGGL(k_step_rhs, dim3(nblocks(H->P.ncell)), dim3(kBlock), 0, H->st, f, c, g,
                           (unsigned)H->P.ncell, 1.0 / dt);
        H->alg_bytes += (double)H->P.ncell * 24;
        int rc;
        if (H->prm.saddle_solver != BLOB_RD_SOLVER_SCHUR) {
            // block FGMRES started from (c^n, previous multipliers or zero)
            if (!warm) launch_fill(H->st, lambda, H->P.N, 0.0);
            const FgOpts o = handle_fg_opts(H, 1.0 / dt);
            char* ws = H->ws + H->P.off_fg;
            rc = H->P.esz == 4 ? fg_entry<float>(H, 1.0 / dt, o, g, c, lambda, ws, stt, true)
                               : fg_entry<double>(H, 1.0 / dt, o, g, c, lambda, ws, stt, true);
        } else {
            const double* lam0 = warm ? lambda : nullptr;
            rc = H->P.esz == 4 ? absorbing_solve<float>(H, 1.0 / dt, g, c, lambda, stt, lam0)
                               : absorbing_solve<double>(H, 1.0 / dt, g, c, lambda, stt, lam0);
        }
        HIPCHK(hipGetLastError());
        return rc;
    });
}

int blob_rd_solve_absorbing(blob_rd_t H, double alpha, const double* f, double* c, double* lambda,
                            blob_rd_stats* stt) {
    if (!H || !f || !c || !lambda) return g_last_error = "null argument", BLOB_RD_EINVAL;
    if (H->P.N <= 0) return g_last_error = "absorbing solve needs at least one blob", BLOB_RD_EINVAL;
    if (!(alpha >= 0.0) || !std::isfinite(alpha)) return g_last_error = "alpha must be >= 0", BLOB_RD_EINVAL;
    if (H->box && H->prm.saddle_solver == BLOB_RD_SOLVER_SCHUR)
        return g_last_error = "absorbing solves in a Dirichlet box need saddle_solver BLOCK", BLOB_RD_EINVAL;
    if (H->prm.saddle_solver != BLOB_RD_SOLVER_SCHUR) {
        blob_rd_saddle_opts o{};
        o.precond = (H->prm.saddle_solver == BLOB_RD_SOLVER_BLOCK_LEARNED && singular(H, alpha))
                        ? BLOB_RD_SADDLE_LEARNED
                        : BLOB_RD_SADDLE_APPROX_SCHUR;
        o.restart = H->P.restart;
        o.maxit = H->prm.max_iter;
        return blob_rd_solve_absorbing_fgmres(H, alpha, &o, f, c, lambda, H->ws + H->P.off_fg, H->P.fg_size, stt);
    }
    return guarded(H, stt, [&]() {
        int rc = H->P.esz == 4 ? absorbing_solve<float>(H, alpha, f, c, lambda, stt)
                               : absorbing_solve<double>(H, alpha, f, c, lambda, stt);
        HIPCHK(hipGetLastError());
        return rc;
    });
}

int blob_rd_interp(blob_rd_t H, const double* c, double* out) {
    if (!H || !c || !out) return g_last_error = "null argument", BLOB_RD_EINVAL;
    return guarded(H, nullptr, [&]() {
        const Plan& P = H->P;
        launch_interp(H->st, c, P.N, P.geom, H->at<int>(P.off_base), H->at<double>(P.off_wts),
                      H->at<int>(P.off_perm), nullptr, nullptr, out, nullptr);
        HIPCHK(hipGetLastError());
        HIPCHK(hipStreamSynchronize(H->st));
        return BLOB_RD_OK;
    });
}

int blob_rd_spread(blob_rd_t H, const double* lambda, double* out) {
    if (!H || !out || (!lambda && H->P.N > 0)) return g_last_error = "null argument", BLOB_RD_EINVAL;
    return guarded(H, nullptr, [&]() {
        spread_to(H, lambda, 0.0, nullptr, out, H->inv_h3(), nullptr);
        HIPCHK(hipGetLastError());
        HIPCHK(hipStreamSynchronize(H->st));
        return BLOB_RD_OK;
    });
}

int blob_rd_apply(blob_rd_t H, double alpha, int with_blobs, const double* x, double* y) {
    if (!H || !x || !y) return g_last_error = "null argument", BLOB_RD_EINVAL;
    if (x == y) return g_last_error = "x and y must not alias", BLOB_RD_EINVAL;
    return guarded(H, nullptr, [&]() {
        const Plan& P = H->P;
        const LevelDims& d = P.lev[0];
        launch_applyA_plain(H->st, x, y, alpha, H->prm.D / (d.h * d.h), d.nx, d.ny, d.nz, H->box);
        if (with_blobs && P.N > 0 && H->has_kappa) blob_term(H, x, y, nullptr);
        HIPCHK(hipGetLastError());
        HIPCHK(hipStreamSynchronize(H->st));
        return BLOB_RD_OK;
    });
}

int blob_rd_vcycle(blob_rd_t H, double alpha, const double* r, double* z) {
    if (!H || !r || !z) return g_last_error = "null argument", BLOB_RD_EINVAL;
    if (!(alpha >= 0.0)) return g_last_error = "alpha must be >= 0", BLOB_RD_EINVAL;
    return guarded(H, nullptr, [&]() {
        const Plan& P = H->P;
        const LevelDims& d = P.lev[0];
        const double* cinv = select_cinv(H, alpha);
        if (P.esz == 4) {
            vcycle<float>(H, alpha, r, nullptr, cinv);
            launch_split_to_nat<float>(H->st, H->at<float>(P.off_lvl[0][0]), H->at<float>(P.off_lvl[0][1]), z, d.nx,
                                       d.ny, d.nz, 0.0);
        } else {
            vcycle<double>(H, alpha, r, nullptr, cinv);
            launch_split_to_nat<double>(H->st, H->at<double>(P.off_lvl[0][0]), H->at<double>(P.off_lvl[0][1]), z,
                                        d.nx, d.ny, d.nz, 0.0);
        }
        HIPCHK(hipGetLastError());
        HIPCHK(hipStreamSynchronize(H->st));
        return BLOB_RD_OK;
    });
}

}  // extern "C"

// ===========================================================================
// Learned preconditioner: network object and configuration hooks.
// ===========================================================================
struct blob_rd_net {
    hipStream_t st = nullptr;
    char* ws = nullptr;
    float* P = nullptr;
    float* m = nullptr;
    float* v = nullptr;
    float* grad = nullptr;
    __bf16* W1b = nullptr;
    __bf16* W2b = nullptr;
    __bf16* w3b = nullptr;
    float* wpart = nullptr;
    int max_waves = 1024;
    int t = 0;
    NetDev dev() const { return NetDev{P, W1b, W2b, w3b}; }
};

namespace {
constexpr int kNetMaxWaves = 1024;
size_t net_bytes() {
    size_t o = 0;
    auto take = [&](size_t b) {
        size_t r = o;
        o = align_up(o + b);
        return r;
    };
    take(4 * (size_t)kNetParams * 4);
    take(64 * 16 * 2);
    take(64 * 64 * 2);
    take(64 * 2);
    take((size_t)kNetMaxWaves * kNetParams * 4);
    return o + 256;
}

PairGeom pair_geom(const blob_rd* H) {
    PairGeom pg{};
    const int n[3] = {H->prm.nx, H->prm.ny, H->prm.nz};
    pg.h = H->prm.h;
    pg.rc = 12.0 * H->prm.h;
    int nc[3];
    for (int a = 0; a < 3; ++a) {
        pg.box[a] = n[a] * H->prm.h;
        nc[a] = (int)std::floor(pg.box[a] / pg.rc);
        if (nc[a] < 3) nc[a] = 1;
    }
    pg.ncx = nc[0];
    pg.ncy = nc[1];
    pg.ncz = nc[2];
    return pg;
}

// Bin blobs into pair-search cells and count pairs per row; int scratch in G_T1.
// Returns nnz; rowptr (N+1) left in the scratch at the returned pointer.
long long pair_count(blob_rd* H, const PairGeom& pg, int** rowptr_out, int** cell_of, int** offsets, int** perm) {
    const Plan& P = H->P;
    const int N = P.N;
    const int nc = pg.ncx * pg.ncy * pg.ncz;
    if (4 * (size_t)N + 3 * (size_t)nc + 2 > 2 * P.ncell) throw Err(BLOB_RD_EINVAL, "too many blobs for the pair scratch");
    int* s = reinterpret_cast<int*>(H->grid(G_T1));
    int* cell = s;
    int* counts = cell + N;
    int* offs = counts + nc;
    int* cursor = offs + nc + 1;
    int* prm = cursor + nc;
    int* cnt = prm + N;
    int* rowptr = cnt + N;
    HIPCHK(hipMemsetAsync(counts, 0, (size_t)nc * 4, H->st));
    HIPCHK(hipMemsetAsync(cursor, 0, (size_t)nc * 4, H->st));
    const double* q = H->at<double>(P.off_q);
    launch_pair_cells(H->st, q, N, pg, cell, counts);
    launch_bin_scan(H->st, counts, nc, offs);
    launch_bin_scatter(H->st, cell, N, offs, cursor, prm);
    launch_bin_sort(H->st, offs, nc, prm);
    launch_pair_count(H->st, q, N, pg, cell, offs, prm, cnt);
    launch_bin_scan(H->st, cnt, N, rowptr);
    int nnz = 0;
    HIPCHK(hipMemcpyAsync(H->hbuf, rowptr + N, sizeof(int), hipMemcpyDeviceToHost, H->st));
    HIPCHK(hipStreamSynchronize(H->st));
    std::memcpy(&nnz, H->hbuf, sizeof(int));
    *rowptr_out = rowptr;
    *cell_of = cell;
    *offsets = offs;
    *perm = prm;
    return nnz;
}

size_t learned_bytes(int N, long long nnz) {
    return align_up((size_t)(N + 1) * 4) + 2 * align_up((size_t)nnz * 4) + align_up((size_t)nnz * 8) +
           align_up((size_t)nnz * 4) + align_up((size_t)N * 4) + 256;
}
}  // namespace

namespace {

// Defined (zero) contents for every multigrid level buffer, before kernels are
// timed on them outside a solve.
void zero_levels(blob_rd* H) {
    const Plan& P = H->P;
    const int L = P.nlev - 1;
    for (int l = 0; l < L; ++l) {
        const size_t hl = (size_t)P.lev[l].hx * P.lev[l].ny * P.lev[l].nz;
        for (int k = 0; k < 5; ++k) HIPCHK(hipMemsetAsync(H->ws + P.off_lvl[l][k], 0, hl * P.esz, H->st));
    }
    HIPCHK(hipMemsetAsync(H->ws + P.off_lvl[L][0], 0, (size_t)P.m * P.esz, H->st));
    HIPCHK(hipMemsetAsync(H->ws + P.off_lvl[L][2], 0, (size_t)P.m * P.esz, H->st));
}

// Levels launched one kernel at a time (above the LDS tail or the dense coarse solve).
int tuned_levels(const blob_rd* H) {
    const int L = H->P.nlev - 1;
    const int t = H->tail_level[H->P.esz == 4 ? 0 : 1];
    return std::max(0, std::min(t, L));
}

const char* const kTuneKind[BLOB_RD_TUNE_KINDS] = {"gs", "resid", "restrict", "prolong"};
const int kTuneCand[4] = {64, 128, 256, 512};

// One launch of tuned kernel `kind` on level l with work-group size bs.
template <typename T>
void tune_launch(blob_rd* H, int l, int kind, int bs) {
    const Plan& P = H->P;
    const int L = P.nlev - 1;
    const bool tail = H->tail_level[sizeof(T) == 4 ? 0 : 1] < L;
    const int cnat = (!tail && l + 1 == L);
    auto lv = [&](int ll, int k) { return H->at<T>(P.off_lvl[ll][k]); };
    const LevelDims& d = P.lev[l];
    const double s = H->prm.D / (d.h * d.h), diag = 6.0 * s;
    switch (kind) {
        case 0: launch_gs<T>(H->st, lv(l, 1), lv(l, 0), lv(l, 3), d.hx, d.ny, d.nz, 1, s, 1.0 / diag, nullptr, bs); break;
        case 1:
            launch_resid_red<T>(H->st, lv(l, 0), lv(l, 1), lv(l, 2), lv(l, 4), d.hx, d.ny, d.nz, s, diag, nullptr, bs);
            break;
        case 2: {
            const LevelDims& c = P.lev[l + 1];
            launch_restrict<T>(H->st, lv(l, 4), d.nx, d.ny, d.nz, lv(l + 1, 2), cnat ? nullptr : lv(l + 1, 3),
                               cnat ? nullptr : lv(l + 1, 0), cnat, 1.0 / (6.0 * H->prm.D / (c.h * c.h)), nullptr, bs);
            break;
        }
        default:
            launch_prolong<T>(H->st, lv(l + 1, 0), cnat ? nullptr : lv(l + 1, 1), cnat, lv(l, 0), lv(l, 1), d.nx, d.ny,
                              d.nz, nullptr, bs);
    }
}

std::string tune_key(const std::string& arch, int esz, const LevelDims& d, int kind) {
    return arch + "|" + (esz == 4 ? "f32" : "f64") + "|" + std::to_string(d.nx) + "x" + std::to_string(d.ny) + "x" +
           std::to_string(d.nz) + "|" + kTuneKind[kind];
}

// The cache file is one flat JSON object of "key": integer pairs, as written below.
std::map<std::string, int> tune_cache_read(const char* path) {
    std::map<std::string, int> m;
    FILE* fp = std::fopen(path, "rb");
    if (!fp) return m;
    std::string txt;
    char buf[4096];
    size_t got;
    while ((got = std::fread(buf, 1, sizeof buf, fp)) > 0) txt.append(buf, got);
    std::fclose(fp);
    size_t i = 0;
    while ((i = txt.find('"', i)) != std::string::npos) {
        const size_t j = txt.find('"', i + 1);
        if (j == std::string::npos) break;
        const std::string key = txt.substr(i + 1, j - i - 1);
        size_t k = txt.find(':', j);
        if (k == std::string::npos) break;
        m[key] = std::atoi(txt.c_str() + k + 1);
        i = txt.find_first_of(",}", k);
        if (i == std::string::npos) break;
    }
    return m;
}

bool tune_cache_write(const char* path, const std::map<std::string, int>& m) {
    const std::string tmp = std::string(path) + ".tmp" + std::to_string((long long)getpid());
    FILE* fp = std::fopen(tmp.c_str(), "wb");
    if (!fp) return false;
    std::fputs("{\n", fp);
    size_t i = 0;
    for (const auto& kv : m) std::fprintf(fp, "  \"%s\": %d%s\n", kv.first.c_str(), kv.second, ++i < m.size() ? "," : "");
    std::fputs("}\n", fp);
    const bool ok = std::fclose(fp) == 0;
    return ok && std::rename(tmp.c_str(), path) == 0;
}

bool valid_block(int v) {
    for (int c : kTuneCand)
        if (v == c) return true;
    return false;
}

void drop_graphs(blob_rd* H) {
    for (auto& g : H->graphs) (void)hipGraphExecDestroy(g.exec);
    H->graphs.clear();
    for (auto& g : H->fg_graphs) (void)hipGraphExecDestroy(g.exec);
    H->fg_graphs.clear();
}

}  // namespace

namespace {

// ===========================================================================
// Lock-step batch executor: the CG iterations of many independent solves run
// as one sequence of batched launches (each launch covers one step, e.g. one
// Gauss-Seidel half-sweep of one level, for every instance through a flat
// block table), captured once as a HIP graph and replayed in rounds. Each
// instance's solver logic (GMRES, set-up, final solves) runs on its own host
// thread and stream; whenever it needs CG iterations it hands them to the
// executor and waits. An instance takes part in a round only when it is gated
// in, and its kernels become no-ops once its done flag is set. Instances that
// solve by the block FGMRES hand the executor their multigrid V-cycles instead:
// a second captured graph runs one V-cycle (entered: level-0 f and the first red
// sweep already written by the instance) for every instance gated into it.
// ===========================================================================
constexpr int kBatchRoundIters = 2;  // CG iterations per graph replay
// a V-cycle round starts when every V-cycle member still solving is waiting, or
// when the first waiter has waited this long (BLOB_RD_VROUND_WAIT_US overrides)
double vround_wait_s() {
    const char* e = std::getenv("BLOB_RD_VROUND_WAIT_US");
    return e ? std::atof(e) * 1e-6 : 300e-6;
}

}  // namespace

// One batched launch's work list: per-instance block counts, and where its
// per-round compacted table lives in the workspace.
struct BatchTable {
    std::vector<unsigned> nb;  // work-group slices per instance (0: not in this launch)
    size_t off = 0;            // byte offset of the BatchTab header in the table region
    unsigned grid = 0;         // fixed grid of the launch
};

struct BatchServer {
    int n = 0, esz = 4;
    double alpha = 0.0;
    std::vector<blob_rd*> hs;
    hipStream_t st = nullptr;
    InstDev* d_inst = nullptr;
    int* d_gate = nullptr;
    int* d_status = nullptr;
    char* d_tabs = nullptr;      // work lists (BatchTab + entries) of every launch
    InstDev* h_inst = nullptr;   // pinned mirrors
    int* h_gate = nullptr;
    int* h_status = nullptr;
    char* h_tabs = nullptr;
    size_t tabs_bytes = 0;
    // work lists: CG direction, stencil, update, closing sweep + dots, interp, spread,
    // then per level sweep/residual/correction and restriction
    std::vector<BatchTable> tabs;
    int Lmax = 0;
    unsigned tail_lds = 0;
    hipGraphExec_t exec = nullptr;
    int rounds = 0;
    // batched V-cycle rounds of the block-FGMRES members: their gate, work lists (the
    // level tables again, compacted for the V-cycle gate), always-open scalars and graph
    std::vector<char> vmem;
    int nvmem = 0;
    int* d_gate_v = nullptr;
    int* h_gate_v = nullptr;
    char* d_tabs_v = nullptr;
    char* h_tabs_v = nullptr;
    size_t tabs_v_bytes = 0;
    std::vector<BatchTable> tabs_v;
    Scalars* d_vsc = nullptr;
    hipGraphExec_t exec_v = nullptr;
    int vrounds = 0;
    long long v_gated = 0;
    long long gated_rounds = 0;  // sum over rounds of gated instances
    double busy_s = 0.0, idle_s = 0.0;
    // coordination
    struct Slot {
        bool vwaiting = false;  // asked for a V-cycle (block-FGMRES members)
        bool vdone = false;     // that V-cycle has run
        std::chrono::steady_clock::time_point vsince;
        bool waiting = false;   // asked for CG iterations
        bool gated = false;     // taking part in rounds
        bool released = false;  // its CG run has ended
        bool dirty = false;     // descriptor changed since the last upload
        bool finished = false;  // its whole solve returned
        int maxit = 0;
        std::condition_variable cv;
    };
    std::vector<Slot> slots;
    std::mutex m;
    std::condition_variable cv;
    std::string fault;  // set when a round fails; waiting instances then fail too
};

namespace {

size_t batch_align(size_t b) { return (b + 255) & ~(size_t)255; }

enum { TAB_DIR = 0, TAB_APPLY, TAB_UPDATE, TAB_DOTS, TAB_INTERP, TAB_SPREAD, TAB_LEVELS };
constexpr unsigned kPersistBlocks = 2048;  // grid of a batched launch (8 work-groups per CU)

size_t batch_tab_bytes(int n) { return batch_align(sizeof(BatchTab) + (size_t)n * sizeof(BatchEntry)); }

size_t batch_bytes(int n) {
    return batch_align((size_t)n * sizeof(InstDev)) + 3 * batch_align((size_t)n * 2 * sizeof(int)) +
           (TAB_LEVELS + 4 * kMaxLevels) * batch_tab_bytes(n) + batch_align((size_t)n * sizeof(Scalars));
}

// Why instance H cannot run its CG iterations in batched launches (empty: it can).
std::string batch_unfit(const blob_rd* H, int esz) {
    const Plan& P = H->P;
    const int L = P.nlev - 1;
    const int t = H->tail_level[P.esz == 4 ? 0 : 1];
    const int VW = 16 / P.esz;
    if ((int)P.esz != esz) return "mixed precisions";
    if (t >= L || t < 1) return "no coarse tail below a per-level finest level";
    for (int l = 0; l < t; ++l) {
        const LevelDims& d = P.lev[l];
        if (d.hx % VW != 0 || (d.nx / 2) % 4 != 0) return "level " + std::to_string(l) + " not vectorizable";
    }
    return "";
}

__global__ void k_batch_status(const InstDev* inst, int n, int* out) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    out[2 * i] = inst[i].sc->done;
    out[2 * i + 1] = inst[i].sc->iters;
}

template <typename T>
void batch_round(BatchServer& B, hipStream_t s) {
    const InstDev* I = B.d_inst;
    const int* G = B.d_gate;
    auto T_ = [&](int k) { return reinterpret_cast<const BatchTab*>(B.d_tabs + B.tabs[k].off); };
    auto grid = [&](int k) { return B.tabs[k].grid; };
    const int LV = TAB_LEVELS, RS = TAB_LEVELS + B.Lmax;
    for (int it = 0; it < kBatchRoundIters; ++it) {
        launchb_cg<T>(s, BCG_DIR, I, G, T_(TAB_DIR), grid(TAB_DIR), B.n);
        launchb_cg<T>(s, BCG_APPLY, I, G, T_(TAB_APPLY), grid(TAB_APPLY), B.n);
        if (grid(TAB_INTERP)) {
            launchb_blob(s, 0, I, G, T_(TAB_INTERP), grid(TAB_INTERP));
            launchb_blob(s, 1, I, G, T_(TAB_SPREAD), grid(TAB_SPREAD));
        }
        launchb_cg<T>(s, BCG_FIN_ALPHA, I, G, nullptr, 0, B.n);
        launchb_cg<T>(s, BCG_UPDATE, I, G, T_(TAB_UPDATE), grid(TAB_UPDATE), B.n);
        launchb_cg<T>(s, BCG_FIN_UPDATE, I, G, nullptr, 0, B.n);
        for (int l = 0; l < B.Lmax; ++l) {
            launchb_mg<T>(s, BMG_GS, I, G, T_(LV + l), grid(LV + l), l, 1, 0);
            launchb_mg<T>(s, BMG_GS, I, G, T_(LV + l), grid(LV + l), l, 0, 0);
            launchb_mg<T>(s, BMG_GS, I, G, T_(LV + l), grid(LV + l), l, 1, 0);
            launchb_mg<T>(s, BMG_RESID, I, G, T_(LV + l), grid(LV + l), l, 0, 0);
            launchb_mg<T>(s, BMG_RESTRICT, I, G, T_(RS + l), grid(RS + l), l, 0, 0);
        }
        launchb_mg<T>(s, BMG_TAIL, I, G, nullptr, B.n, 0, 0, B.tail_lds);
        for (int l = B.Lmax - 1; l >= 0; --l) {
            launchb_mg<T>(s, BMG_PROLONG, I, G, T_(LV + l), grid(LV + l), l, 0, 0);
            launchb_mg<T>(s, BMG_GS, I, G, T_(LV + l), grid(LV + l), l, 1, 0);
            launchb_mg<T>(s, BMG_GS, I, G, T_(LV + l), grid(LV + l), l, 0, 0);
            launchb_mg<T>(s, BMG_GS, I, G, T_(LV + l), grid(LV + l), l, 1, 0);
            if (l == 0)
                launchb_mg<T>(s, BMG_GS_DOTS, I, G, T_(TAB_DOTS), grid(TAB_DOTS), 0, 0, 0);
            else
                launchb_mg<T>(s, BMG_GS, I, G, T_(LV + l), grid(LV + l), l, 0, 0);
        }
        launchb_cg<T>(s, BCG_FIN_BETA, I, G, nullptr, 0, B.n);
    }
    hipLaunchKernelGGL(k_batch_status, dim3((B.n + 63) / 64), dim3(64), 0, s, I, B.n, B.d_status);
}

// One entered V-cycle (level-0 f and the first red sweep written by the instance) of
// every instance gated into the V-cycle rounds: the per-level launches of the CG
// round's preconditioner, closing with a plain red sweep.
template <typename T>
void batch_round_v(BatchServer& B, hipStream_t s) {
    const InstDev* I = B.d_inst;
    const int* G = B.d_gate_v;
    auto T_ = [&](int k) { return reinterpret_cast<const BatchTab*>(B.d_tabs_v + B.tabs_v[k].off); };
    auto grid = [&](int k) { return B.tabs_v[k].grid; };
    const int LV = 0, RS = B.Lmax;
    for (int l = 0; l < B.Lmax; ++l) {
        launchb_mg<T>(s, BMG_GS, I, G, T_(LV + l), grid(LV + l), l, 1, 0);
        launchb_mg<T>(s, BMG_GS, I, G, T_(LV + l), grid(LV + l), l, 0, 0);
        launchb_mg<T>(s, BMG_GS, I, G, T_(LV + l), grid(LV + l), l, 1, 0);
        launchb_mg<T>(s, BMG_RESID, I, G, T_(LV + l), grid(LV + l), l, 0, 0);
        launchb_mg<T>(s, BMG_RESTRICT, I, G, T_(RS + l), grid(RS + l), l, 0, 0);
    }
    launchb_mg<T>(s, BMG_TAIL, I, G, nullptr, B.n, 0, 0, B.tail_lds);
    for (int l = B.Lmax - 1; l >= 0; --l) {
        launchb_mg<T>(s, BMG_PROLONG, I, G, T_(LV + l), grid(LV + l), l, 0, 0);
        launchb_mg<T>(s, BMG_GS, I, G, T_(LV + l), grid(LV + l), l, 1, 0);
        launchb_mg<T>(s, BMG_GS, I, G, T_(LV + l), grid(LV + l), l, 0, 0);
        launchb_mg<T>(s, BMG_GS, I, G, T_(LV + l), grid(LV + l), l, 1, 0);
        launchb_mg<T>(s, BMG_GS, I, G, T_(LV + l), grid(LV + l), l, 0, 0);
    }
}

// Work lists of the round: the gated instances' slices, each starting at a
// multiple of 8 virtual blocks (a slot keeps the XCD of its solo launch).
void fill_tabs(const std::vector<BatchTable>& tabs, const int* gate, char* h_tabs, int n) {
    for (const BatchTable& t : tabs) {
        BatchTab* h = reinterpret_cast<BatchTab*>(h_tabs + t.off);
        BatchEntry* e = reinterpret_cast<BatchEntry*>(h + 1);
        unsigned g = 0;
        int k = 0;
        for (int i = 0; i < n; ++i) {
            if (!gate[i] || !t.nb[i]) continue;
            e[k++] = BatchEntry{g, t.nb[i], i, 0};
            g += (t.nb[i] + 7u) & ~7u;
        }
        h->total = g;
        h->n = k;
    }
}
void batch_fill_tabs(BatchServer& B) { fill_tabs(B.tabs, B.h_gate, B.h_tabs, B.n); }

// Descriptor of instance H for CG iterations with operator alpha (x set per CG run).
void batch_describe(BatchServer& B, int i, blob_rd* H, bool blobs) {
    const Plan& P = H->P;
    InstDev& D = B.h_inst[i];
    std::memset(&D, 0, sizeof(InstDev));
    const int L = P.nlev - 1;
    const int t = H->tail_level[P.esz == 4 ? 0 : 1];
    D.sc = B.vmem[i] ? B.d_vsc + i : H->sc();  // V-cycle members: a done flag that stays 0
    D.part = H->part();
    D.x = H->grid(G_U);
    D.r = H->grid(G_R);
    D.p = H->grid(G_P);
    D.q = H->grid(G_Q);
    D.alpha = B.alpha;
    D.nx = P.lev[0].nx;
    D.ny = P.lev[0].ny;
    D.nz = P.lev[0].nz;
    D.nlev = P.nlev;
    D.t = t;
    for (int l = 0; l <= L; ++l) {
        for (int k = 0; k < 5; ++k) D.lv[l][k] = H->ws + P.off_lvl[l][k];
        D.lnx[l] = P.lev[l].nx;
        D.lny[l] = P.lev[l].ny;
        D.lnz[l] = P.lev[l].nz;
        D.ls[l] = H->prm.D / (P.lev[l].h * P.lev[l].h);
        D.ldiag[l] = B.alpha + 6.0 * D.ls[l];
    }
    const unsigned npair = (unsigned)(D.nx / 2) * D.ny * D.nz;
    D.np_apply = D.np_update = (int)red_blocks(npair);
    D.np_dots = (int)nblocks((size_t)(P.lev[0].hx / (16 / P.esz)) * D.ny * D.nz);
    D.blobs = blobs ? 1 : 0;
    D.N = P.N;
    D.geom = P.geom;
    D.base = H->at<int>(P.off_base);
    D.wts = H->at<double>(P.off_wts);
    D.offsets = H->at<int>(P.off_offsets);
    D.perm = H->at<int>(P.off_perm);
    D.kappa = H->at<double>(P.off_kappa);
    D.jx = H->nv(0);
    D.mu = H->nv(1);
    D.inv_h3 = H->inv_h3();
    D.ntouched = H->ntouched;
    D.tcell = H->at<int>(P.off_tcell);
    D.tptr = H->at<int>(P.off_tptr);
    D.tblob = H->at<int>(P.off_tblob);
    D.tw = H->at<double>(P.off_tw);
    D.cinv = select_cinv(H, B.alpha);
    D.tail = P.esz == 4 ? make_tail<float>(H, t, B.alpha) : make_tail<double>(H, t, B.alpha);
}

void batch_setup(BatchServer& B, char* ws, size_t ws_bytes, const int32_t* kind) {
    const int n = B.n;
    char* o = ws;
    B.d_inst = reinterpret_cast<InstDev*>(o);
    o += batch_align((size_t)n * sizeof(InstDev));
    B.d_gate = reinterpret_cast<int*>(o);
    o += batch_align((size_t)n * 2 * sizeof(int));
    B.d_status = reinterpret_cast<int*>(o);
    o += batch_align((size_t)n * 2 * sizeof(int));
    B.d_gate_v = reinterpret_cast<int*>(o);
    o += batch_align((size_t)n * 2 * sizeof(int));
    B.d_vsc = reinterpret_cast<Scalars*>(o);
    o += batch_align((size_t)n * sizeof(Scalars));
    B.d_tabs = o;
    B.d_tabs_v = o + (TAB_LEVELS + 2 * kMaxLevels) * batch_tab_bytes(n);
    (void)ws_bytes;
    HIPCHK(hipMemsetAsync(B.d_vsc, 0, (size_t)n * sizeof(Scalars), B.st));
    HIPCHK(hipHostMalloc((void**)&B.h_inst, (size_t)n * sizeof(InstDev), hipHostMallocDefault));
    HIPCHK(hipHostMalloc((void**)&B.h_gate, (size_t)n * 2 * sizeof(int), hipHostMallocDefault));
    HIPCHK(hipHostMalloc((void**)&B.h_status, (size_t)n * 2 * sizeof(int), hipHostMallocDefault));
    HIPCHK(hipHostMalloc((void**)&B.h_gate_v, (size_t)n * 2 * sizeof(int), hipHostMallocDefault));
    std::memset(B.h_gate_v, 0, (size_t)n * 2 * sizeof(int));
    B.Lmax = 0;
    for (int i = 0; i < n; ++i) {
        blob_rd* H = B.hs[i];
        const bool blobs = kind[i] == 0 && H->P.N > 0 && H->has_kappa;
        batch_describe(B, i, H, blobs);
        HIPCHK(hipStreamSynchronize(H->st));  // coarse inverse uploads
        B.Lmax = std::max(B.Lmax, B.h_inst[i].t);
        B.tail_lds = std::max(B.tail_lds, B.h_inst[i].tail.lds_bytes);
        B.h_gate[i] = 0;
    }
    const int VW = 16 / B.esz;
    auto npair = [&](int i) { const InstDev& D = B.h_inst[i]; return (size_t)(D.nx / 2) * D.ny * D.nz; };
    auto nv = [&](int i, int l) {
        const InstDev& D = B.h_inst[i];
        return (size_t)(D.lnx[l] / 2 / VW) * D.lny[l] * D.lnz[l];
    };
    B.tabs.assign(TAB_LEVELS + 2 * B.Lmax, BatchTable{});
    for (auto& t : B.tabs) t.nb.assign(n, 0u);
    for (int i = 0; i < n; ++i) {
        const InstDev& D = B.h_inst[i];
        B.tabs[TAB_DIR].nb[i] = nblocks(npair(i));
        B.tabs[TAB_APPLY].nb[i] = red_blocks(npair(i));
        B.tabs[TAB_UPDATE].nb[i] = red_blocks(npair(i));
        B.tabs[TAB_DOTS].nb[i] = nblocks(nv(i, 0));
        if (D.blobs) {
            B.tabs[TAB_INTERP].nb[i] = (unsigned)((D.N + kBlock / 64 - 1) / (kBlock / 64));
            B.tabs[TAB_SPREAD].nb[i] = nblocks((size_t)D.ntouched);
        }
        for (int l = 0; l < D.t; ++l) {
            B.tabs[TAB_LEVELS + l].nb[i] = nblocks(nv(i, l));
            B.tabs[TAB_LEVELS + B.Lmax + l].nb[i] =
                nblocks((size_t)(D.lnx[l] / 2 / 4) * (D.lny[l] / 2) * (D.lnz[l] / 2));
        }
    }
    const size_t tb = batch_tab_bytes(n);
    for (size_t k = 0; k < B.tabs.size(); ++k) {
        BatchTable& t = B.tabs[k];
        t.off = k * tb;
        unsigned all = 0;
        for (unsigned v : t.nb) all += (v + 7u) & ~7u;
        t.grid = std::min(all, kPersistBlocks);
    }
    B.tabs_bytes = B.tabs.size() * tb;
    HIPCHK(hipHostMalloc((void**)&B.h_tabs, B.tabs_bytes, hipHostMallocDefault));
    std::memset(B.h_tabs, 0, B.tabs_bytes);
    // the V-cycle rounds' copies of the level tables (sweep/residual/correction, restriction)
    B.tabs_v.assign(2 * B.Lmax, BatchTable{});
    for (int k = 0; k < 2 * B.Lmax; ++k) {
        B.tabs_v[k] = B.tabs[TAB_LEVELS + k];
        B.tabs_v[k].off = (size_t)k * tb;
    }
    B.tabs_v_bytes = std::max<size_t>(B.tabs_v.size() * tb, tb);
    HIPCHK(hipHostMalloc((void**)&B.h_tabs_v, B.tabs_v_bytes, hipHostMallocDefault));
    std::memset(B.h_tabs_v, 0, B.tabs_v_bytes);
    HIPCHK(hipMemcpyAsync(B.d_tabs, B.h_tabs, B.tabs_bytes, hipMemcpyHostToDevice, B.st));
    HIPCHK(hipMemcpyAsync(B.d_inst, B.h_inst, (size_t)n * sizeof(InstDev), hipMemcpyHostToDevice, B.st));
    HIPCHK(hipMemcpyAsync(B.d_gate, B.h_gate, (size_t)n * sizeof(int), hipMemcpyHostToDevice, B.st));
    HIPCHK(hipStreamSynchronize(B.st));
    if (B.esz == 4) HIPCHK(tail_set_lds_batched<float>(std::max<unsigned>(B.tail_lds, 1)));
    else HIPCHK(tail_set_lds_batched<double>(std::max<unsigned>(B.tail_lds, 1)));
    hipStream_t cap;
    HIPCHK(hipStreamCreateWithFlags(&cap, hipStreamNonBlocking));
    HIPCHK(hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal));
    if (B.esz == 4) batch_round<float>(B, cap);
    else batch_round<double>(B, cap);
    hipGraph_t graph;
    HIPCHK(hipStreamEndCapture(cap, &graph));
    HIPCHK(hipGraphInstantiate(&B.exec, graph, nullptr, nullptr, 0));
    (void)hipGraphDestroy(graph);
    if (B.nvmem) {
        HIPCHK(hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal));
        if (B.esz == 4) batch_round_v<float>(B, cap);
        else batch_round_v<double>(B, cap);
        HIPCHK(hipStreamEndCapture(cap, &graph));
        HIPCHK(hipGraphInstantiate(&B.exec_v, graph, nullptr, nullptr, 0));
        (void)hipGraphDestroy(graph);
    }
    (void)hipStreamDestroy(cap);
}

void batch_teardown(BatchServer& B) {
    if (B.exec) (void)hipGraphExecDestroy(B.exec);
    if (B.exec_v) (void)hipGraphExecDestroy(B.exec_v);
    if (B.h_gate_v) (void)hipHostFree(B.h_gate_v);
    if (B.h_tabs_v) (void)hipHostFree(B.h_tabs_v);
    B.exec_v = nullptr;
    B.h_gate_v = nullptr;
    B.h_tabs_v = nullptr;
    if (B.h_inst) (void)hipHostFree(B.h_inst);
    if (B.h_gate) (void)hipHostFree(B.h_gate);
    if (B.h_status) (void)hipHostFree(B.h_status);
    if (B.h_tabs) (void)hipHostFree(B.h_tabs);
    B.exec = nullptr;
    B.h_inst = nullptr;
    B.h_gate = B.h_status = nullptr;
    B.h_tabs = nullptr;
}

// Instance side: hand this CG run (x, at most maxit iterations) to the executor
// and wait until it has converged, failed or used its iterations.
void batch_run_cg(blob_rd* H, double* x, int maxit, bool blobs, double alpha) {
    BatchServer& B = *H->batch;
    const int i = H->batch_slot;
    std::unique_lock<std::mutex> lk(B.m);
    if (!B.fault.empty()) throw Err(BLOB_RD_EDEVICE, "batch executor: " + B.fault);
    // the batched launches were laid out for one operator per instance
    if (alpha != B.alpha || (blobs ? 1 : 0) != B.h_inst[i].blobs)
        throw Err(BLOB_RD_EINVAL, "batch executor: CG operator differs from the one the batch was laid out for");
    BatchServer::Slot& S = B.slots[i];
    if (B.h_inst[i].x != x) {
        B.h_inst[i].x = x;
        S.dirty = true;
    }
    S.maxit = maxit;
    S.released = false;
    S.waiting = true;
    B.cv.notify_all();
    S.cv.wait(lk, [&] { return S.released || !B.fault.empty(); });
    if (!B.fault.empty() && !S.released) throw Err(BLOB_RD_EDEVICE, "batch executor: " + B.fault);
}

// Instance side: one entered V-cycle of H's levels in the executor's next V-cycle round
// (after H's own work so far, through its event); returns once that round has run.
void batch_run_vcycle(blob_rd* H) {
    BatchServer& B = *H->batch;
    const int i = H->batch_slot;
    HIPCHK(hipEventRecord(H->batch_ev, H->st));
    std::unique_lock<std::mutex> lk(B.m);
    if (!B.fault.empty()) throw Err(BLOB_RD_EDEVICE, "batch executor: " + B.fault);
    BatchServer::Slot& S = B.slots[i];
    S.vdone = false;
    S.vwaiting = true;
    S.vsince = std::chrono::steady_clock::now();
    B.cv.notify_all();
    S.cv.wait(lk, [&] { return S.vdone || !B.fault.empty(); });
    if (!B.fault.empty() && !S.vdone) throw Err(BLOB_RD_EDEVICE, "batch executor: " + B.fault);
}

// Executor side: rounds of the captured graph for the gated instances until
// every instance's solve has returned.
void batch_serve(BatchServer& B) {
    using clk = std::chrono::steady_clock;
    const auto vwait = std::chrono::duration_cast<clk::duration>(std::chrono::duration<double>(vround_wait_s()));
    for (;;) {
        std::vector<int> upload, vgated;
        const auto w0 = clk::now();
        bool any = false;
        {
            std::unique_lock<std::mutex> lk(B.m);
            // CG work starts a round at once; V-cycle requests wait for the other V-cycle
            // members still solving (they ask at nearly the same points) or for a deadline
            auto ready = [&](clk::time_point* deadline) {
                bool cg = false, all_done = true, vany = false, vall = true;
                clk::time_point first = clk::time_point::max();
                for (int i = 0; i < B.n; ++i) {
                    const BatchServer::Slot& S = B.slots[i];
                    cg = cg || S.waiting || S.gated;
                    all_done = all_done && S.finished;
                    if (!B.vmem[i] || S.finished) continue;
                    if (S.vwaiting) {
                        vany = true;
                        first = std::min(first, S.vsince);
                    } else {
                        vall = false;
                    }
                }
                if (vany) *deadline = first + vwait;
                return cg || all_done || (vany && (vall || clk::now() >= *deadline));
            };
            for (;;) {
                clk::time_point deadline = clk::time_point::max();
                if (ready(&deadline)) break;
                if (deadline == clk::time_point::max()) B.cv.wait(lk);
                else B.cv.wait_until(lk, deadline);
            }
            for (int i = 0; i < B.n; ++i) {
                BatchServer::Slot& S = B.slots[i];
                if (S.waiting) {
                    S.waiting = false;
                    S.gated = true;
                    B.h_gate[i] = 1;
                    if (S.dirty) upload.push_back(i);
                    S.dirty = false;
                }
                B.h_gate_v[i] = 0;
                if (S.vwaiting) {
                    S.vwaiting = false;
                    B.h_gate_v[i] = 1;
                    vgated.push_back(i);
                }
                any = any || S.gated;
            }
            if (!any && vgated.empty()) return;  // every solve has returned
            if (any) batch_fill_tabs(B);
            if (!vgated.empty()) fill_tabs(B.tabs_v, B.h_gate_v, B.h_tabs_v, B.n);
        }
        const auto w1 = clk::now();
        B.idle_s += std::chrono::duration<double>(w1 - w0).count();
        for (int i = 0; i < B.n; ++i) B.gated_rounds += B.h_gate[i];
        try {
            if (!vgated.empty()) {
                for (int i : vgated) HIPCHK(hipStreamWaitEvent(B.st, B.hs[i]->batch_ev, 0));
                HIPCHK(hipMemcpyAsync(B.d_gate_v, B.h_gate_v, (size_t)B.n * sizeof(int), hipMemcpyHostToDevice,
                                      B.st));
                HIPCHK(hipMemcpyAsync(B.d_tabs_v, B.h_tabs_v, B.tabs_v_bytes, hipMemcpyHostToDevice, B.st));
                HIPCHK(hipGraphLaunch(B.exec_v, B.st));
            }
            if (any) {
                for (int i : upload)
                    HIPCHK(hipMemcpyAsync(B.d_inst + i, B.h_inst + i, sizeof(InstDev), hipMemcpyHostToDevice, B.st));
                HIPCHK(hipMemcpyAsync(B.d_gate, B.h_gate, (size_t)B.n * sizeof(int), hipMemcpyHostToDevice, B.st));
                HIPCHK(hipMemcpyAsync(B.d_tabs, B.h_tabs, B.tabs_bytes, hipMemcpyHostToDevice, B.st));
                HIPCHK(hipGraphLaunch(B.exec, B.st));
                HIPCHK(hipMemcpyAsync(B.h_status, B.d_status, (size_t)B.n * 2 * sizeof(int),
                                      hipMemcpyDeviceToHost, B.st));
            }
            HIPCHK(hipStreamSynchronize(B.st));
        } catch (const Err& e) {
            std::lock_guard<std::mutex> lk(B.m);
            B.fault = e.what();
            for (auto& S : B.slots) S.cv.notify_all();
            return;
        }
        if (any) ++B.rounds;
        if (!vgated.empty()) {
            ++B.vrounds;
            B.v_gated += (long long)vgated.size();
        }
        B.busy_s += std::chrono::duration<double>(clk::now() - w1).count();
        std::lock_guard<std::mutex> lk(B.m);
        for (int i : vgated) {
            B.slots[i].vdone = true;
            B.slots[i].cv.notify_all();
        }
        for (int i = 0; i < B.n; ++i) {
            BatchServer::Slot& S = B.slots[i];
            if (!S.gated) continue;
            if (B.h_status[2 * i] || B.h_status[2 * i + 1] >= S.maxit) {
                S.gated = false;
                B.h_gate[i] = 0;
                S.released = true;
                S.cv.notify_all();
            }
        }
    }
}

}  // namespace

extern "C" {

size_t blob_rd_net_workspace_bytes(void) { return net_bytes(); }

int blob_rd_net_create(void* workspace, size_t bytes, void* stream, blob_rd_net_t* out) {
    if (!out || !workspace) return g_last_error = "null argument", BLOB_RD_EINVAL;
    if (bytes < net_bytes()) return g_last_error = "net workspace too small", BLOB_RD_ENOMEM;
    blob_rd_net* N = new blob_rd_net();
    N->st = (hipStream_t)stream;
    N->ws = (char*)(((uintptr_t)workspace + 255) & ~(uintptr_t)255);
    size_t o = 0;
    auto take = [&](size_t b) {
        size_t r = o;
        o = align_up(o + b);
        return N->ws + r;
    };
    char* base = take(4 * (size_t)kNetParams * 4);
    N->P = (float*)base;
    N->m = N->P + kNetParams;
    N->v = N->m + kNetParams;
    N->grad = N->v + kNetParams;
    N->W1b = (__bf16*)take(64 * 16 * 2);
    N->W2b = (__bf16*)take(64 * 64 * 2);
    N->w3b = (__bf16*)take(64 * 2);
    N->wpart = (float*)take((size_t)kNetMaxWaves * kNetParams * 4);
    N->max_waves = kNetMaxWaves;
    if (hipMemsetAsync(N->P, 0, 4 * (size_t)kNetParams * 4, N->st) != hipSuccess) {
        delete N;
        return g_last_error = "hipMemsetAsync failed", BLOB_RD_EDEVICE;
    }
    launch_net_pack(N->st, N->P, N->W1b, N->W2b, N->w3b);
    *out = N;
    return BLOB_RD_OK;
}

int blob_rd_net_destroy(blob_rd_net_t N) {
    delete N;
    return BLOB_RD_OK;
}

int blob_rd_net_set_params(blob_rd_net_t N, const float* params) {
    if (!N || !params) return g_last_error = "null argument", BLOB_RD_EINVAL;
    try {
        HIPCHK(hipMemcpyAsync(N->P, params, (size_t)kNetParams * 4, hipMemcpyDeviceToDevice, N->st));
        HIPCHK(hipMemsetAsync(N->m, 0, 3 * (size_t)kNetParams * 4, N->st));  // m, v, grad
        N->t = 0;
        launch_net_pack(N->st, N->P, N->W1b, N->W2b, N->w3b);
        HIPCHK(hipGetLastError());
        HIPCHK(hipStreamSynchronize(N->st));
    } catch (const Err& e) {
        return fail(nullptr, e);
    }
    return BLOB_RD_OK;
}

int blob_rd_net_get_params(blob_rd_net_t N, float* params) {
    if (!N || !params) return g_last_error = "null argument", BLOB_RD_EINVAL;
    if (hipMemcpyAsync(params, N->P, (size_t)kNetParams * 4, hipMemcpyDeviceToDevice, N->st) != hipSuccess ||
        hipStreamSynchronize(N->st) != hipSuccess)
        return g_last_error = "copy failed", BLOB_RD_EDEVICE;
    return BLOB_RD_OK;
}

int blob_rd_net_zero_grad(blob_rd_net_t N) {
    if (!N) return g_last_error = "null argument", BLOB_RD_EINVAL;
    return hipMemsetAsync(N->grad, 0, (size_t)kNetParams * 4, N->st) == hipSuccess ? BLOB_RD_OK : BLOB_RD_EDEVICE;
}

int blob_rd_net_get_grad(blob_rd_net_t N, float* grad) {
    if (!N || !grad) return g_last_error = "null argument", BLOB_RD_EINVAL;
    if (hipMemcpyAsync(grad, N->grad, (size_t)kNetParams * 4, hipMemcpyDeviceToDevice, N->st) != hipSuccess ||
        hipStreamSynchronize(N->st) != hipSuccess)
        return g_last_error = "copy failed", BLOB_RD_EDEVICE;
    return BLOB_RD_OK;
}

int blob_rd_net_adam_step(blob_rd_net_t N, float lr) {
    if (!N || !(lr > 0.f)) return g_last_error = "bad argument", BLOB_RD_EINVAL;
    N->t += 1;
    launch_adam(N->st, N->P, N->m, N->v, N->grad, lr, 0.9f, 0.999f, 1e-8f, N->t);
    launch_net_pack(N->st, N->P, N->W1b, N->W2b, N->w3b);
    return hipGetLastError() == hipSuccess ? BLOB_RD_OK : BLOB_RD_EDEVICE;
}

}  // extern "C"

namespace {

// Pair list of the handle's blobs and W from network Nt into buf (256-byte slack
// included in learned_bytes); with buf null only *needed is set.
int precond_build_into(blob_rd* H, blob_rd_net* Nt, void* buf, size_t bytes, size_t* needed) {
    const int N = H->P.N;
    const PairGeom pg = pair_geom(H);
    int *rowptr_s, *cell, *offs, *prm;
    const long long nnz = pair_count(H, pg, &rowptr_s, &cell, &offs, &prm);
    const size_t need = learned_bytes(N, nnz);
    if (needed) *needed = need;
    if (!buf) return BLOB_RD_OK;
    if (bytes < need) throw Err(BLOB_RD_ENOMEM, "precond buffer smaller than the size reported");
    char* b = (char*)(((uintptr_t)buf + 255) & ~(uintptr_t)255);
    if (b + need - 256 > (char*)buf + bytes) throw Err(BLOB_RD_ENOMEM, "precond buffer misaligned/too small");
    // captured block-FGMRES steps read the previous W's buffers
    HIPCHK(hipStreamSynchronize(H->st));
    for (auto& g : H->fg_graphs) (void)hipGraphExecDestroy(g.exec);
    H->fg_graphs.clear();
    auto& L = H->lrn;
    L.rowptr = (int*)b;
    b += align_up((size_t)(N + 1) * 4);
    L.col = (int*)b;
    b += align_up((size_t)nnz * 4);
    L.rowidx = (int*)b;
    b += align_up((size_t)nnz * 4);
    L.val = (double*)b;
    b += align_up((size_t)nnz * 8);
    L.dg = (float*)b;
    b += align_up((size_t)nnz * 4);
    L.nu = (float*)b;
    L.nnz = nnz;
    L.pg = pg;
    L.pg.nu = L.nu;
    const double* q = H->at<double>(H->P.off_q);
    HIPCHK(hipMemcpyAsync(L.rowptr, rowptr_s, (size_t)(N + 1) * 4, hipMemcpyDeviceToDevice, H->st));
    launch_pair_fill(H->st, q, N, pg, cell, offs, prm, L.rowptr, L.col, L.rowidx);
    launch_rowidx(H->st, L.rowptr, N, L.rowidx);
    launch_pair_nu(H->st, q, L.pg, L.rowptr, L.col, N, L.nu);
    // the network's stream ordering: make sure its weights are current
    HIPCHK(hipStreamSynchronize(Nt->st));
    launch_net_assemble(H->st, q, L.pg, Nt->dev(), L.col, L.rowidx, nnz, H->prm.D * H->prm.h,
                        4.0 * M_PI * 1.255, L.val);
    int* bad = reinterpret_cast<int*>(H->dsc() + 40);
    launch_count_bad(H->st, L.val, nnz, bad);
    HIPCHK(hipMemcpyAsync(H->hbuf, bad, sizeof(int), hipMemcpyDeviceToHost, H->st));
    HIPCHK(hipStreamSynchronize(H->st));
    int nbad = 0;
    std::memcpy(&nbad, H->hbuf, sizeof(int));
    L.bad = nbad != 0;
    L.ready = true;
    H->own_w = Nt == H->own_net;
    HIPCHK(hipGetLastError());
    return BLOB_RD_OK;
}

}  // namespace

extern "C" {

int blob_rd_precond_build(blob_rd_t H, blob_rd_net_t Nt, void* buf, size_t bytes, size_t* needed) {
    if (!H || !Nt) return g_last_error = "null argument", BLOB_RD_EINVAL;
    if (H->P.N <= 0) return g_last_error = "no blobs", BLOB_RD_EINVAL;
    if (H->box) return g_last_error = "the learned preconditioner is for the periodic cell", BLOB_RD_EINVAL;
    return guarded(H, nullptr, [&]() { return precond_build_into(H, Nt, buf, bytes, needed); });
}

int blob_rd_precond_apply(blob_rd_t H, const double* r, double* z) {
    if (!H || !r || !z) return g_last_error = "null argument", BLOB_RD_EINVAL;
    if (!H->lrn.ready) return g_last_error = "learned preconditioner not built", BLOB_RD_EINVAL;
    return guarded(H, nullptr, [&]() {
        precond_apply(H, r, z);
        HIPCHK(hipGetLastError());
        HIPCHK(hipStreamSynchronize(H->st));
        return BLOB_RD_OK;
    });
}

size_t blob_rd_coarse_bytes(blob_rd_t H, int32_t m2max) {
    // |m|^2 <= 16 gives 256 columns, the most the level takes; larger m2max are refused
    // before the wave vectors are enumerated
    if (!H || H->P.N <= 0 || m2max < 1 || m2max > 16) return g_last_error = "bad argument", (size_t)0;
    const int K = (int)coarse_modes(m2max).size() / 3 * 2;
    return coarse_layout(H->P.N, K, nullptr, nullptr);
}

int blob_rd_coarse_build(blob_rd_t H, double alpha, int32_t m2max, double inner_rtol, void* buf, size_t bytes,
                         int32_t* ncols) {
    if (!H || !buf) return g_last_error = "null argument", BLOB_RD_EINVAL;
    if (H->P.N <= 0) return g_last_error = "no blobs", BLOB_RD_EINVAL;
    if (H->box) return g_last_error = "the Fourier coarse level is for the periodic cell", BLOB_RD_EINVAL;
    if (H->batch) return g_last_error = "the handle is in a batch", BLOB_RD_EINVAL;
    if (!(alpha >= 0.0) || !std::isfinite(alpha)) return g_last_error = "alpha must be finite and >= 0", BLOB_RD_EINVAL;
    if (inner_rtol == 0.0) inner_rtol = 1e-6;
    if (!(inner_rtol > 0.0 && inner_rtol < 1.0)) return g_last_error = "inner_rtol must be in (0, 1)", BLOB_RD_EINVAL;
    if (m2max < 1 || m2max > 16) return g_last_error = "m2max must be in [1, 16]", BLOB_RD_EINVAL;
    const std::vector<int> mv = coarse_modes(m2max);
    const int K = (int)mv.size() / 3 * 2;
    if (K > kMaxCoarseCols)
        return g_last_error = "more than " + std::to_string(kMaxCoarseCols) + " coarse columns", BLOB_RD_EINVAL;
    if (K > H->P.N - (alpha == 0.0 ? 1 : 0))
        return g_last_error = "more coarse columns than the blobs' mean-free dimension", BLOB_RD_EINVAL;
    if (bytes < coarse_layout(H->P.N, K, nullptr, nullptr)) return g_last_error = "coarse buffer too small", BLOB_RD_ENOMEM;
    return guarded(H, nullptr, [&]() {
        if (H->P.esz == 4) coarse_build<float>(H, alpha, mv, inner_rtol, static_cast<char*>(buf));
        else coarse_build<double>(H, alpha, mv, inner_rtol, static_cast<char*>(buf));
        if (ncols) *ncols = K;
        return BLOB_RD_OK;
    });
}

int blob_rd_coarse_clear(blob_rd_t H) {
    if (!H) return g_last_error = "null argument", BLOB_RD_EINVAL;
    return guarded(H, nullptr, [&]() {
        drop_fg_graphs(H);
        H->crs = blob_rd::Coarse{};
        return BLOB_RD_OK;
    });
}

int blob_rd_coarse_apply(blob_rd_t H, const double* r, double* z) {
    if (!H || !r || !z || r == z) return g_last_error = "bad argument", BLOB_RD_EINVAL;
    if (!H->crs.ready) return g_last_error = "coarse level not built", BLOB_RD_EINVAL;
    const bool use_w = H->prm.schur_precond == BLOB_RD_PRECOND_LEARNED && H->crs.alpha == 0.0 && H->lrn.ready &&
                       !H->lrn.bad;
    return guarded(H, nullptr, [&]() {
        coarse_apply(H, use_w, r, z);
        HIPCHK(hipGetLastError());
        HIPCHK(hipStreamSynchronize(H->st));
        return BLOB_RD_OK;
    });
}

int blob_rd_precond_csr(blob_rd_t H, int64_t* nnz, int32_t* rowptr, int32_t* col, double* val) {
    if (!H || !nnz) return g_last_error = "null argument", BLOB_RD_EINVAL;
    if (!H->lrn.ready) return g_last_error = "learned preconditioner not built", BLOB_RD_EINVAL;
    *nnz = H->lrn.nnz;
    try {
        const int N = H->P.N;
        if (rowptr) HIPCHK(hipMemcpyAsync(rowptr, H->lrn.rowptr, (size_t)(N + 1) * 4, hipMemcpyDeviceToDevice, H->st));
        if (col) HIPCHK(hipMemcpyAsync(col, H->lrn.col, (size_t)H->lrn.nnz * 4, hipMemcpyDeviceToDevice, H->st));
        if (val) HIPCHK(hipMemcpyAsync(val, H->lrn.val, (size_t)H->lrn.nnz * 8, hipMemcpyDeviceToDevice, H->st));
        HIPCHK(hipStreamSynchronize(H->st));
    } catch (const Err& e) {
        return fail(H, e);
    }
    return BLOB_RD_OK;
}

int blob_rd_precond_loss_grad(blob_rd_t H, blob_rd_net_t Nt, const double* X, const double* Y, int32_t S,
                              double* loss) {
    if (!H || !Nt || !X || !Y || S <= 0 || S > 64) return g_last_error = "bad argument", BLOB_RD_EINVAL;
    if (!H->lrn.ready) return g_last_error = "learned preconditioner not built", BLOB_RD_EINVAL;
    return guarded(H, nullptr, [&]() {
        const int N = H->P.N;
        auto& L = H->lrn;
        hipStream_t st = H->st;
        if ((size_t)2 * S * N + 64 > H->P.ncell) throw Err(BLOB_RD_EINVAL, "too many samples for this grid");
        double* RP = H->grid(G_T2);
        double* YP = RP + (size_t)S * N;
        double* coef = YP + (size_t)S * N;
        double lsum = 0.0;
        std::vector<double> cf(S);
        for (int s = 0; s < S; ++s) {
            double* yp = YP + (size_t)s * N;
            double* rp = RP + (size_t)s * N;
            launch_nvec_copy_scale(st, Y + (size_t)s * N, yp, N, 1.0, 0.0);
            launch_nvec_project(st, yp, N);
            launch_spmv(st, L.rowptr, L.col, L.val, yp, rp, N);
            launch_nvec_project(st, rp, N);
            launch_axpby(st, rp, X + (size_t)s * N, N, 1.0, -1.0);   // res = P W P y - x
            launch_nvec_sums(st, rp, nullptr, N, H->dsc());
            launch_nvec_sums(st, X + (size_t)s * N, nullptr, N, H->dsc() + 3);
            sync_read(H, H->hbuf, H->dsc(), 6 * 8);
            const double rr = H->hbuf[1], xx = H->hbuf[4];
            if (!(xx > 0.0)) throw Err(BLOB_RD_EINVAL, "zero sample x");
            lsum += rr / xx / S;
            cf[s] = 2.0 / (S * xx);
            launch_nvec_project(st, rp, N);
        }
        HIPCHK(hipMemcpyAsync(coef, cf.data(), (size_t)S * 8, hipMemcpyHostToDevice, st));
        launch_entry_grad(st, L.rowidx, L.col, L.nnz, RP, YP, coef, S, N, 0.5 * H->prm.D * H->prm.h, L.dg);
        HIPCHK(hipStreamSynchronize(Nt->st));
        const int nw = launch_net_backward(st, H->at<double>(H->P.off_q), L.pg, Nt->dev(), L.col, L.rowidx, L.nnz,
                                           L.dg, Nt->wpart, Nt->max_waves);
        launch_grad_reduce(st, Nt->wpart, nw, Nt->grad);
        HIPCHK(hipGetLastError());
        HIPCHK(hipStreamSynchronize(st));
        if (loss) *loss = lsum;
        return BLOB_RD_OK;
    });
}

}  // extern "C"

namespace {

// The inference blob of the network: bfloat16 weights and float32 biases, in the
// order of the float32 parameter vector.
struct BlobPart {
    int off_param, count;
    bool bf16;
};
constexpr BlobPart kBlobParts[6] = {{kOffW1, 64 * kNetFeat, true}, {kOffB1, 64, false}, {kOffW2, 4096, true},
                                    {kOffB2, 64, false}, {kOffW3, 64, true},  {kOffB3, 1, false}};

float bf16_to_float(uint16_t b) {
    const uint32_t u = (uint32_t)b << 16;
    float f;
    std::memcpy(&f, &u, 4);
    return f;
}

// round to nearest, ties to even (NaN stays a quiet NaN)
uint16_t float_to_bf16(float f) {
    uint32_t u;
    std::memcpy(&u, &f, 4);
    if ((u & 0x7f800000u) == 0x7f800000u && (u & 0x007fffffu)) return (uint16_t)((u >> 16) | 0x40);
    u += 0x7fffu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}

void blob_to_params(const unsigned char* blob, std::vector<float>& P) {
    P.assign(kNetParams, 0.f);
    size_t o = 0;
    for (const BlobPart& part : kBlobParts) {
        for (int k = 0; k < part.count; ++k) {
            if (part.bf16) {
                uint16_t b;
                std::memcpy(&b, blob + o, 2);
                P[part.off_param + k] = bf16_to_float(b);
                o += 2;
            } else {
                std::memcpy(&P[part.off_param + k], blob + o, 4);
                o += 4;
            }
        }
    }
}

void params_to_blob(const std::vector<float>& P, unsigned char* blob) {
    size_t o = 0;
    for (const BlobPart& part : kBlobParts) {
        for (int k = 0; k < part.count; ++k) {
            if (part.bf16) {
                const uint16_t b = float_to_bf16(P[part.off_param + k]);
                std::memcpy(blob + o, &b, 2);
                o += 2;
            } else {
                std::memcpy(blob + o, &P[part.off_param + k], 4);
                o += 4;
            }
        }
    }
}

// W of the handle's own network into the handle's learned region.
void own_build(blob_rd* H) {
    size_t need = 0;
    precond_build_into(H, H->own_net, nullptr, 0, &need);
    if (need > H->P.lrn_size)
        throw Err(BLOB_RD_ENOMEM, "more blob pairs within 12h than the handle reserves (" +
                                      std::to_string(BLOB_RD_LEARNED_ROW_CAP) + " per blob on average)");
    precond_build_into(H, H->own_net, H->ws + H->P.off_lrn, H->P.lrn_size, &need);
}

int need_own_net(blob_rd* H) {
    if (!H->own_net) {
        g_last_error = "the handle holds no network: create it with schur_precond = LEARNED or saddle_solver = "
                       "BLOCK_LEARNED, a periodic domain and at least one blob";
        return BLOB_RD_EINVAL;
    }
    return BLOB_RD_OK;
}

}  // namespace

extern "C" {

int blob_rd_precond_set_weights(blob_rd_t H, const void* blob, size_t bytes) {
    if (!H || !blob) return g_last_error = "null argument", BLOB_RD_EINVAL;
    if (bytes != BLOB_RD_PRECOND_BLOB_BYTES)
        return g_last_error = "weight blob must be BLOB_RD_PRECOND_BLOB_BYTES bytes", BLOB_RD_EINVAL;
    if (int rc = need_own_net(H)) return rc;
    return guarded(H, nullptr, [&]() {
        std::vector<float> P;
        blob_to_params(static_cast<const unsigned char*>(blob), P);
        blob_rd_net* Nt = H->own_net;
        HIPCHK(hipMemcpyAsync(Nt->P, P.data(), (size_t)kNetParams * 4, hipMemcpyHostToDevice, Nt->st));
        HIPCHK(hipMemsetAsync(Nt->m, 0, 3 * (size_t)kNetParams * 4, Nt->st));  // m, v, grad
        Nt->t = 0;
        launch_net_pack(Nt->st, Nt->P, Nt->W1b, Nt->W2b, Nt->w3b);
        HIPCHK(hipGetLastError());
        HIPCHK(hipStreamSynchronize(Nt->st));
        own_build(H);
        return BLOB_RD_OK;
    });
}

int blob_rd_precond_get_weights(blob_rd_t H, void* blob, size_t bytes) {
    if (!H || !blob) return g_last_error = "null argument", BLOB_RD_EINVAL;
    if (bytes != BLOB_RD_PRECOND_BLOB_BYTES)
        return g_last_error = "weight blob must be BLOB_RD_PRECOND_BLOB_BYTES bytes", BLOB_RD_EINVAL;
    if (int rc = need_own_net(H)) return rc;
    return guarded(H, nullptr, [&]() {
        std::vector<float> P(kNetParams);
        HIPCHK(hipMemcpyAsync(P.data(), H->own_net->P, (size_t)kNetParams * 4, hipMemcpyDeviceToHost,
                              H->own_net->st));
        HIPCHK(hipStreamSynchronize(H->own_net->st));
        params_to_blob(P, static_cast<unsigned char*>(blob));
        return BLOB_RD_OK;
    });
}

int blob_rd_precond_train_step(blob_rd_t H, const void* batch_desc, float lr, float* loss) {
    if (!H || !batch_desc) return g_last_error = "null argument", BLOB_RD_EINVAL;
    if (!(lr > 0.f) || !std::isfinite(lr)) return g_last_error = "learning rate must be positive", BLOB_RD_EINVAL;
    if (int rc = need_own_net(H)) return rc;
    const blob_rd_train_batch* b = static_cast<const blob_rd_train_batch*>(batch_desc);
    if (!b->x || !b->y || b->n_samples <= 0 || b->n_samples > 64)
        return g_last_error = "training batch needs 1..64 samples and device x, y", BLOB_RD_EINVAL;
    return guarded(H, nullptr, [&]() {
        blob_rd_net* Nt = H->own_net;
        if (!H->lrn.ready || !H->own_w) own_build(H);
        HIPCHK(hipMemsetAsync(Nt->grad, 0, (size_t)kNetParams * 4, Nt->st));
        double l = 0.0;
        int rc = blob_rd_precond_loss_grad(H, Nt, b->x, b->y, b->n_samples, &l);
        if (rc != BLOB_RD_OK) throw Err(rc, g_last_error);
        if (blob_rd_net_adam_step(Nt, lr) != BLOB_RD_OK) throw Err(BLOB_RD_EDEVICE, "Adam step failed");
        own_build(H);  // the handle's W follows the updated weights
        if (loss) *loss = (float)l;
        return BLOB_RD_OK;
    });
}

int blob_rd_schur_apply(blob_rd_t H, double alpha, const double* x, double* y, double inner_rtol) {
    if (!H || !x || !y || H->P.N <= 0) return g_last_error = "bad argument", BLOB_RD_EINVAL;
    if (!(alpha >= 0.0) || !(inner_rtol > 0.0)) return g_last_error = "bad alpha or tolerance", BLOB_RD_EINVAL;
    return guarded(H, nullptr, [&]() {
        if (H->P.esz == 4) schur_apply<float>(H, alpha, x, y, inner_rtol);
        else schur_apply<double>(H, alpha, x, y, inner_rtol);
        HIPCHK(hipGetLastError());
        HIPCHK(hipStreamSynchronize(H->st));
        return BLOB_RD_OK;
    });
}

int blob_rd_solve_streams(blob_rd_t* hs, int32_t n, const int32_t* kind, double alpha, const double* const* f,
                          double* const* c, double* const* lambda, int32_t threads, blob_rd_stats* stats) {
    if (!hs || !kind || !f || !c || n < 0 || threads <= 0) return g_last_error = "bad argument", BLOB_RD_EINVAL;
    for (int i = 0; i < n; ++i) {
        if (!hs[i] || !f[i] || !c[i] || (kind[i] == 1 && (!lambda || !lambda[i])) || (kind[i] != 0 && kind[i] != 1))
            return g_last_error = "bad instance " + std::to_string(i), BLOB_RD_EINVAL;
        for (int j = 0; j < i; ++j)
            if (hs[j] == hs[i]) return g_last_error = "a handle appears twice in the batch", BLOB_RD_EINVAL;
    }
    // largest grids first for load balance
    std::vector<int> order(n);
    for (int i = 0; i < n; ++i) order[i] = i;
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return hs[a]->P.ncell > hs[b]->P.ncell; });
    std::vector<int> rcs(n, 0);
    std::vector<std::string> errs(n);
    std::atomic<int> next(0);
    auto worker = [&]() {
        for (;;) {
            const int k = next.fetch_add(1);
            if (k >= n) return;
            const int i = order[k];
            blob_rd_stats* si = stats ? &stats[i] : nullptr;
            rcs[i] = kind[i] == 0 ? blob_rd_solve_reactive(hs[i], alpha, f[i], c[i], si)
                                  : blob_rd_solve_absorbing(hs[i], alpha, f[i], c[i], lambda[i], si);
            if (rcs[i] < 0) errs[i] = g_last_error;
        }
    };
    const int nt = std::max(1, std::min<int>(threads, n));
    std::vector<std::thread> pool;
    for (int t = 1; t < nt; ++t) pool.emplace_back(worker);
    worker();
    for (auto& t : pool) t.join();
    int rc = BLOB_RD_OK;
    for (int i = 0; i < n; ++i)
        if (rcs[i] < 0) {
            g_last_error = "instance " + std::to_string(i) + ": " + errs[i];
            return rcs[i];
        }
    for (int i = 0; i < n; ++i)
        if (rcs[i] == BLOB_RD_ENOTCONV) rc = BLOB_RD_ENOTCONV;
    return rc;
}

int blob_rd_time_kernel(blob_rd_t H, int kernel, int reps, double* avg_ms, double* bytes) {
    if (!H || !avg_ms || !bytes || reps <= 0) return g_last_error = "bad argument", BLOB_RD_EINVAL;
    const bool cold = (kernel & BLOB_RD_KERNEL_COLD) != 0;
    kernel &= ~BLOB_RD_KERNEL_COLD;
    if (kernel < 0 || kernel > 6) return g_last_error = "unknown kernel id", BLOB_RD_EINVAL;
    return guarded(H, nullptr, [&]() {
        const Plan& P = H->P;
        const LevelDims& d = P.lev[0];
        const double alpha = 0.0, s = H->prm.D / (d.h * d.h), diag = alpha + 6.0 * s;
        const double* cinv = select_cinv(H, alpha);
        // a box handle times its own kernels (the box forms of the same steps)
        const bool box = H->box;
        BoxCoef bdg0, binv0, binv1;
        box_coefs(H, 0, alpha, &bdg0, &binv0);
        box_coefs(H, 1, alpha, nullptr, &binv1);
        auto gs_any = [&](auto* uc, const auto* uo, const auto* fc) {
            typedef std::remove_const_t<std::remove_pointer_t<decltype(uo)>> TT;
            if (box) launch_gs_box<TT>(H->st, uc, uo, fc, d.nx, d.ny, d.nz, 1, s, binv0, nullptr);
            else launch_gs<TT>(H->st, uc, uo, fc, d.hx, d.ny, d.nz, 1, s, 1.0 / diag, nullptr);
        };
        zero_levels(H);
        HIPCHK(hipMemsetAsync(H->grid(G_P), 0, P.ncell * 8, H->st));
        HIPCHK(hipMemsetAsync(H->grid(G_R), 0, P.ncell * 8, H->st));
        hipEvent_t e0, e1;
        HIPCHK(hipEventCreate(&e0));
        HIPCHK(hipEventCreate(&e1));
        auto one = [&]() {
            const bool f32 = P.esz == 4;
            const LevelDims& c = P.lev[1];
            const int cnat = P.nlev == 2;
            const size_t half_bytes = (size_t)d.hx * d.ny * d.nz * P.esz;
            switch (kernel) {
                case BLOB_RD_KERNEL_STREAM:
                    launch_stream_add(H->st, H->at<char>(P.off_lvl[0][0]), H->at<char>(P.off_lvl[0][3]),
                                      H->at<char>(P.off_lvl[0][1]), half_bytes);
                    break;
                case BLOB_RD_KERNEL_GS:
                    if (f32) gs_any(H->at<float>(P.off_lvl[0][1]), H->at<float>(P.off_lvl[0][0]),
                                    H->at<float>(P.off_lvl[0][3]));
                    else gs_any(H->at<double>(P.off_lvl[0][1]), H->at<double>(P.off_lvl[0][0]),
                                H->at<double>(P.off_lvl[0][3]));
                    break;
                case BLOB_RD_KERNEL_STENCIL: {
                    unsigned npp = 0;
                    launch_applyA2(H->st, H->grid(G_P), H->grid(G_Q), alpha, s, d.nx, d.ny, d.nz, H->part(), nullptr,
                                   &npp, box);
                    break;
                }
                case BLOB_RD_KERNEL_STENCIL_PLAIN:
                    launch_applyA_plain(H->st, H->grid(G_P), H->grid(G_Q), alpha, s, d.nx, d.ny, d.nz, box);
                    break;
                case BLOB_RD_KERNEL_RESTRICT:
                    if (box && f32) {
                        launch_resid_red_box<float>(H->st, H->at<float>(P.off_lvl[0][0]),
                                                    H->at<float>(P.off_lvl[0][1]), H->at<float>(P.off_lvl[0][2]),
                                                    H->at<float>(P.off_lvl[0][4]), d.nx, d.ny, d.nz, s, bdg0, nullptr);
                        launch_restrict_box<float>(H->st, H->at<float>(P.off_lvl[0][4]), d.nx, d.ny, d.nz,
                                                   H->at<float>(P.off_lvl[1][2]),
                                                   cnat ? nullptr : H->at<float>(P.off_lvl[1][3]),
                                                   cnat ? nullptr : H->at<float>(P.off_lvl[1][0]), cnat, binv1,
                                                   nullptr);
                    } else if (box) {
                        launch_resid_red_box<double>(H->st, H->at<double>(P.off_lvl[0][0]),
                                                     H->at<double>(P.off_lvl[0][1]), H->at<double>(P.off_lvl[0][2]),
                                                     H->at<double>(P.off_lvl[0][4]), d.nx, d.ny, d.nz, s, bdg0,
                                                     nullptr);
                        launch_restrict_box<double>(H->st, H->at<double>(P.off_lvl[0][4]), d.nx, d.ny, d.nz,
                                                    H->at<double>(P.off_lvl[1][2]),
                                                    cnat ? nullptr : H->at<double>(P.off_lvl[1][3]),
                                                    cnat ? nullptr : H->at<double>(P.off_lvl[1][0]), cnat, binv1,
                                                    nullptr);
                    } else if (f32) {
                        launch_resid_red<float>(H->st, H->at<float>(P.off_lvl[0][0]), H->at<float>(P.off_lvl[0][1]),
                                                H->at<float>(P.off_lvl[0][2]), H->at<float>(P.off_lvl[0][4]), d.hx,
                                                d.ny, d.nz, s, diag, nullptr);
                        launch_restrict<float>(H->st, H->at<float>(P.off_lvl[0][4]), d.nx,
                                               d.ny, d.nz, H->at<float>(P.off_lvl[1][2]),
                                               cnat ? nullptr : H->at<float>(P.off_lvl[1][3]),
                                               cnat ? nullptr : H->at<float>(P.off_lvl[1][0]), cnat,
                                               1.0 / (alpha + 6.0 * H->prm.D / (c.h * c.h)), nullptr);
                    } else {
                        launch_resid_red<double>(H->st, H->at<double>(P.off_lvl[0][0]), H->at<double>(P.off_lvl[0][1]),
                                                 H->at<double>(P.off_lvl[0][2]), H->at<double>(P.off_lvl[0][4]), d.hx,
                                                 d.ny, d.nz, s, diag, nullptr);
                        launch_restrict<double>(H->st, H->at<double>(P.off_lvl[0][4]),
                                                d.nx, d.ny, d.nz, H->at<double>(P.off_lvl[1][2]),
                                                cnat ? nullptr : H->at<double>(P.off_lvl[1][3]),
                                                cnat ? nullptr : H->at<double>(P.off_lvl[1][0]), cnat,
                                                1.0 / (alpha + 6.0 * H->prm.D / (c.h * c.h)), nullptr);
                    }
                    break;
                case BLOB_RD_KERNEL_PROLONG:
                    if (box && f32) launch_prolong_red_box<float>(H->st, H->at<float>(P.off_lvl[1][0]),
                                                                  cnat ? nullptr : H->at<float>(P.off_lvl[1][1]), cnat,
                                                                  H->at<float>(P.off_lvl[0][0]), d.nx, d.ny, d.nz,
                                                                  nullptr);
                    else if (box) launch_prolong_red_box<double>(H->st, H->at<double>(P.off_lvl[1][0]),
                                                                 cnat ? nullptr : H->at<double>(P.off_lvl[1][1]), cnat,
                                                                 H->at<double>(P.off_lvl[0][0]), d.nx, d.ny, d.nz,
                                                                 nullptr);
                    else if (f32) launch_prolong<float>(H->st, H->at<float>(P.off_lvl[1][0]),
                                                   cnat ? nullptr : H->at<float>(P.off_lvl[1][1]), cnat,
                                                   H->at<float>(P.off_lvl[0][0]), H->at<float>(P.off_lvl[0][1]), d.nx,
                                                   d.ny, d.nz, nullptr);
                    else launch_prolong<double>(H->st, H->at<double>(P.off_lvl[1][0]),
                                                cnat ? nullptr : H->at<double>(P.off_lvl[1][1]), cnat,
                                                H->at<double>(P.off_lvl[0][0]), H->at<double>(P.off_lvl[0][1]), d.nx,
                                                d.ny, d.nz, nullptr);
                    break;
                default:
                    if (f32) vcycle<float>(H, alpha, H->grid(G_R), nullptr, cinv);
                    else vcycle<double>(H, alpha, H->grid(G_R), nullptr, cinv);
            }
        };
        float ms = 0.f;
        if (cold && (kernel == BLOB_RD_KERNEL_GS || kernel == BLOB_RD_KERNEL_STENCIL ||
                     kernel == BLOB_RD_KERNEL_STREAM || kernel == BLOB_RD_KERNEL_STENCIL_PLAIN)) {
            // Back-to-back launches rotating over independent buffer sets carved
            // from the eight FP64 grid vectors (> 256 MB in all), so no launch
            // finds its data in the last-level cache; event overhead is spread
            // over all the launches.
            const bool gs = kernel != BLOB_RD_KERNEL_STENCIL && kernel != BLOB_RD_KERNEL_STENCIL_PLAIN;
            const bool plain = kernel == BLOB_RD_KERNEL_STENCIL_PLAIN;
            const bool stream = kernel == BLOB_RD_KERNEL_STREAM;
            const size_t abytes = gs ? (size_t)d.hx * d.ny * d.nz * P.esz : P.ncell * 8;
            const size_t per_grid = (P.ncell * 8) / abytes;
            std::vector<char*> arr;
            for (int g = 0; g < 8; ++g) {
                HIPCHK(hipMemsetAsync(H->grid(g), 0, P.ncell * 8, H->st));
                for (size_t k = 0; k < per_grid; ++k) arr.push_back(reinterpret_cast<char*>(H->grid(g)) + k * abytes);
            }
            const int per_set = gs ? 3 : 2;
            const int nset = (int)(arr.size() / per_set);
            auto launch_set = [&](int k) {
                char** a = &arr[(size_t)k * per_set];
                if (stream) {
                    launch_stream_add(H->st, a[1], a[2], a[0], abytes);
                } else if (plain) {
                    launch_applyA_plain(H->st, (const double*)a[0], (double*)a[1], alpha, s, d.nx, d.ny, d.nz, box);
                } else if (!gs) {
                    unsigned npp = 0;
                    launch_applyA2(H->st, (const double*)a[0], (double*)a[1], alpha, s, d.nx, d.ny, d.nz, H->part(),
                                   nullptr, &npp, box);
                } else if (P.esz == 4) {
                    gs_any((float*)a[0], (const float*)a[1], (const float*)a[2]);
                } else {
                    gs_any((double*)a[0], (const double*)a[1], (const double*)a[2]);
                }
            };
            for (int k = 0; k < nset; ++k) launch_set(k);  // first touch
            HIPCHK(hipEventRecord(e0, H->st));
            for (int i = 0; i < reps; ++i) launch_set(i % nset);
            HIPCHK(hipEventRecord(e1, H->st));
            HIPCHK(hipEventSynchronize(e1));
            HIPCHK(hipEventElapsedTime(&ms, e0, e1));
        } else if (cold) {
            one();  // warm
            // Evict the 256 MB Infinity Cache before every timed launch by streaming
            // through >= 512 MB of the workspace's FP64 scratch vectors.
            double* flush = H->grid(G_T1);
            const size_t fl = std::min<size_t>(3 * P.ncell, (size_t)96 << 20);  // doubles (G_T1, G_T2, G_P2 are adjacent)
            for (int i = 0; i < reps; ++i) {
                launch_axpby(H->st, flush, flush + fl / 2, fl / 2, 0.5, 0.5);
                HIPCHK(hipEventRecord(e0, H->st));
                one();
                HIPCHK(hipEventRecord(e1, H->st));
                HIPCHK(hipEventSynchronize(e1));
                float t = 0.f;
                HIPCHK(hipEventElapsedTime(&t, e0, e1));
                ms += t;
            }
        } else {
            one();  // warm
            HIPCHK(hipEventRecord(e0, H->st));
            for (int i = 0; i < reps; ++i) one();
            HIPCHK(hipEventRecord(e1, H->st));
            HIPCHK(hipEventSynchronize(e1));
            HIPCHK(hipEventElapsedTime(&ms, e0, e1));
        }
        (void)hipEventDestroy(e0);
        (void)hipEventDestroy(e1);
        *avg_ms = (double)ms / reps;
        const double n = (double)P.ncell, e = (double)P.esz;
        switch (kernel) {
            case BLOB_RD_KERNEL_GS: *bytes = n * 0.5 * e * 3; break;              // other colour, f, own colour
            case BLOB_RD_KERNEL_STREAM: *bytes = n * 0.5 * e * 3; break;          // a, b in, out
            case BLOB_RD_KERNEL_STENCIL: *bytes = n * 16; break;                 // read x, write y (FP64)
            case BLOB_RD_KERNEL_STENCIL_PLAIN: *bytes = n * 16; break;
            case BLOB_RD_KERNEL_RESTRICT: *bytes = n * e * 2.5 + n / 8 * e * 1.5; break;  // red u, black u, red f; red r write+read; coarse f, u
            case BLOB_RD_KERNEL_PROLONG: *bytes = n * e + n / 8 * e; break;  // red u read+write, coarse read
            default: {
                double b = 0.0;
                for (int l = 0; l + 1 < P.nlev; ++l)
                    b += n / (double)(1 << (3 * l)) * e * (kPreRestrictBytes + kProlongPostBytes);
                *bytes = b + n * (8 + 1.5 * e);  // + entry: FP64 residual in, f and the first red sweep out
            }
        }
        HIPCHK(hipGetLastError());
        return BLOB_RD_OK;
    });
}

int blob_rd_tune_levels(blob_rd_t H) {
    if (!H) return g_last_error = "null handle", BLOB_RD_EINVAL;
    return tuned_levels(H);
}

int blob_rd_get_tuning(blob_rd_t H, int32_t* table, int32_t n_entries) {
    if (!H || !table) return g_last_error = "bad argument", BLOB_RD_EINVAL;
    const int nl = tuned_levels(H);
    if (n_entries < nl * BLOB_RD_TUNE_KINDS) return g_last_error = "table too small", BLOB_RD_EINVAL;
    for (int l = 0; l < nl; ++l)
        for (int k = 0; k < BLOB_RD_TUNE_KINDS; ++k) table[l * BLOB_RD_TUNE_KINDS + k] = H->bs[l][k];
    return BLOB_RD_OK;
}

int blob_rd_set_tuning(blob_rd_t H, const int32_t* table, int32_t n_entries) {
    if (!H || !table) return g_last_error = "bad argument", BLOB_RD_EINVAL;
    const int nl = tuned_levels(H);
    if (n_entries < nl * BLOB_RD_TUNE_KINDS) return g_last_error = "table too small", BLOB_RD_EINVAL;
    for (int i = 0; i < nl * BLOB_RD_TUNE_KINDS; ++i)
        if (!valid_block(table[i]))
            return g_last_error = "work-group size " + std::to_string(table[i]) + " is not 64, 128, 256 or 512",
                   BLOB_RD_EINVAL;
    for (int l = 0; l < nl; ++l)
        for (int k = 0; k < BLOB_RD_TUNE_KINDS; ++k) H->bs[l][k] = table[l * BLOB_RD_TUNE_KINDS + k];
    drop_graphs(H);
    return BLOB_RD_OK;
}

int blob_rd_autotune(blob_rd_t H, int32_t reps, const char* cache_path, int32_t* timed) {
    if (!H || reps <= 0) return g_last_error = "bad argument", BLOB_RD_EINVAL;
    if (H->box) return g_last_error = "launch tuning covers the periodic multigrid kernels", BLOB_RD_EINVAL;
    if (!cache_path) cache_path = std::getenv("BLOB_RD_TUNE_CACHE");
    return guarded(H, nullptr, [&]() {
        const Plan& P = H->P;
        const int nl = tuned_levels(H);
        int dev = 0;
        HIPCHK(hipGetDevice(&dev));
        hipDeviceProp_t prop;
        HIPCHK(hipGetDeviceProperties(&prop, dev));
        std::string arch = prop.gcnArchName;
        arch = arch.substr(0, arch.find(':'));
        std::map<std::string, int> cache;
        if (cache_path) cache = tune_cache_read(cache_path);
        int ntimed = 0;
        hipEvent_t e0 = nullptr, e1 = nullptr;
        for (int l = 0; l < nl; ++l) {
            int found[BLOB_RD_TUNE_KINDS];
            bool all = true;
            for (int k = 0; k < BLOB_RD_TUNE_KINDS; ++k) {
                auto it = cache.find(tune_key(arch, P.esz, P.lev[l], k));
                found[k] = (it != cache.end() && valid_block(it->second)) ? it->second : 0;
                all = all && found[k];
            }
            if (all) {
                for (int k = 0; k < BLOB_RD_TUNE_KINDS; ++k) H->bs[l][k] = found[k];
                continue;
            }
            if (!e0) {
                HIPCHK(hipEventCreate(&e0));
                HIPCHK(hipEventCreate(&e1));
                zero_levels(H);
            }
            for (int k = 0; k < BLOB_RD_TUNE_KINDS; ++k) {
                float best = 0.f, def = 0.f;
                int pick = kBlock;
                for (int c : kTuneCand) {
                    auto one = [&]() {
                        if (P.esz == 4) tune_launch<float>(H, l, k, c);
                        else tune_launch<double>(H, l, k, c);
                    };
                    one();
                    HIPCHK(hipEventRecord(e0, H->st));
                    for (int r = 0; r < reps; ++r) one();
                    HIPCHK(hipEventRecord(e1, H->st));
                    HIPCHK(hipEventSynchronize(e1));
                    float ms = 0.f;
                    HIPCHK(hipEventElapsedTime(&ms, e0, e1));
                    if (c == kBlock) def = ms;
                    if (best == 0.f || ms < best) best = ms, pick = c;
                }
                if (best > 0.97f * def) pick = kBlock;
                H->bs[l][k] = pick;
                cache[tune_key(arch, P.esz, P.lev[l], k)] = pick;
            }
            ++ntimed;
        }
        if (e0) (void)hipEventDestroy(e0);
        if (e1) (void)hipEventDestroy(e1);
        HIPCHK(hipGetLastError());
        drop_graphs(H);
        if (timed) *timed = ntimed;
        if (cache_path && ntimed > 0 && !tune_cache_write(cache_path, cache)) {
            g_last_error = std::string("cannot write tuning cache ") + cache_path;
            return BLOB_RD_EINVAL;
        }
        return BLOB_RD_OK;
    });
}

size_t blob_rd_batch_workspace_bytes(int32_t n) { return n > 0 ? batch_bytes(n) + 256 : 0; }

int blob_rd_solve_batched(blob_rd_t* hs, int32_t n, const int32_t* kind, double alpha, const double* const* f,
                          double* const* c, double* const* lambda, int64_t lockstep_max_cells, int32_t threads,
                          void* workspace, size_t workspace_bytes, void* stream, blob_rd_stats* stats) {
    if (!hs || !kind || !f || !c || n <= 0 || threads < 0) return g_last_error = "bad argument", BLOB_RD_EINVAL;
    if (!workspace || workspace_bytes < blob_rd_batch_workspace_bytes(n))
        return g_last_error = "batch workspace missing or smaller than blob_rd_batch_workspace_bytes()",
               BLOB_RD_ENOMEM;
    for (int i = 0; i < n; ++i) {
        if (!hs[i] || !f[i] || !c[i] || (kind[i] == 1 && (!lambda || !lambda[i])) || (kind[i] != 0 && kind[i] != 1))
            return g_last_error = "bad instance " + std::to_string(i), BLOB_RD_EINVAL;
        for (int j = 0; j < i; ++j)
            if (hs[j] == hs[i]) return g_last_error = "a handle appears twice in the batch", BLOB_RD_EINVAL;
        if (hs[i]->batch) return g_last_error = "instance " + std::to_string(i) + " is in another batch", BLOB_RD_EINVAL;
    }
    // Members of the lock-step launches: grids up to lockstep_max_cells whose
    // levels fit the batched kernels, in the first member's precision. The
    // others run their CG iterations on their own streams meanwhile.
    // Block-FGMRES absorbing instances join as V-cycle members: their multigrid cycles
    // run in the batched V-cycle rounds.
    std::vector<int> member, mkind;
    std::vector<char> vmem;
    int esz = 0;
    for (int i = 0; i < n; ++i) {
        const blob_rd* H = hs[i];
        const bool block = kind[i] == 1 && H->prm.saddle_solver != BLOB_RD_SOLVER_SCHUR;
        if (lockstep_max_cells > 0 && (int64_t)H->P.ncell > lockstep_max_cells) continue;
        if (H->box) continue;  // the batched kernels are the periodic ones
        if (!batch_unfit(H, esz ? esz : (int)H->P.esz).empty()) continue;
        esz = (int)H->P.esz;
        member.push_back(i);
        mkind.push_back(kind[i]);
        vmem.push_back(block ? 1 : 0);
    }
    BatchServer B;
    B.n = (int)member.size();
    B.esz = esz ? esz : 4;
    B.alpha = alpha;
    B.vmem = vmem;
    for (char v : vmem) B.nvmem += v;
    for (int i : member) B.hs.push_back(hs[i]);
    B.st = (hipStream_t)stream;
    B.slots = std::vector<BatchServer::Slot>(B.n);
    if (B.n) {
        uintptr_t base = ((uintptr_t)workspace + 255) & ~(uintptr_t)255;
        try {
            batch_setup(B, reinterpret_cast<char*>(base), workspace_bytes - (base - (uintptr_t)workspace),
                        mkind.data());
        } catch (const Err& e) {
            batch_teardown(B);
            g_last_error = e.what();
            return e.code;
        }
        for (int k = 0; k < B.n; ++k) {
            blob_rd* H = hs[member[k]];
            if (B.vmem[k] && !H->batch_ev &&
                hipEventCreateWithFlags(&H->batch_ev, hipEventDisableTiming) != hipSuccess) {
                batch_teardown(B);
                g_last_error = "event creation failed";
                return BLOB_RD_EDEVICE;
            }
        }
        for (int k = 0; k < B.n; ++k) {
            hs[member[k]]->batch = &B;
            hs[member[k]]->batch_slot = k;
            hs[member[k]]->batch_v = B.vmem[k] != 0;
        }
    }
    std::vector<int> rcs(n, 0), slot_of(n, -1);
    for (int k = 0; k < B.n; ++k) slot_of[member[k]] = k;
    std::vector<std::string> errs(n);
    // the instances outside the lock-step launches share `threads` concurrent solves
    std::mutex qm;
    std::condition_variable qcv;
    int running = 0;
    const int cap = threads > 0 ? threads : n;
    std::vector<std::thread> th;
    th.reserve(n);
    for (int i = 0; i < n; ++i)
        th.emplace_back([&, i]() {
            const bool outside = slot_of[i] < 0;
            if (outside) {
                std::unique_lock<std::mutex> lk(qm);
                qcv.wait(lk, [&] { return running < cap; });
                ++running;
            }
            blob_rd_stats* si = stats ? &stats[i] : nullptr;
            rcs[i] = kind[i] == 0 ? blob_rd_solve_reactive(hs[i], alpha, f[i], c[i], si)
                                  : blob_rd_solve_absorbing(hs[i], alpha, f[i], c[i], lambda[i], si);
            if (rcs[i] < 0) errs[i] = g_last_error;
            if (outside) {
                std::lock_guard<std::mutex> lk(qm);
                --running;
                qcv.notify_all();
            } else {
                std::lock_guard<std::mutex> lk(B.m);
                B.slots[slot_of[i]].finished = true;
                B.cv.notify_all();
            }
        });
    const auto t0 = std::chrono::steady_clock::now();
    if (B.n) batch_serve(B);
    for (auto& t : th) t.join();
    if (std::getenv("BLOB_RD_LOG"))
        std::fprintf(stderr, "[blob_rd] batched solve: %d instances (%d in lock-step launches, %d of them by V-cycle "
                     "rounds), %.1f ms, %d CG rounds, %d V-cycle rounds (%.1f ms running, %.1f ms waiting for "
                     "instances), %.1f instances per CG round, %.1f per V-cycle round\n", n, B.n, B.nvmem,
                     1e3 * std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count(), B.rounds,
                     B.vrounds, 1e3 * B.busy_s, 1e3 * B.idle_s, B.rounds ? (double)B.gated_rounds / B.rounds : 0.0,
                     B.vrounds ? (double)B.v_gated / B.vrounds : 0.0);
    for (int k = 0; k < B.n; ++k) {
        hs[member[k]]->batch = nullptr;
        hs[member[k]]->batch_slot = -1;
        hs[member[k]]->batch_v = false;
    }
    batch_teardown(B);
    for (int i = 0; i < n; ++i)
        if (rcs[i] < 0) {
            g_last_error = "instance " + std::to_string(i) + ": " + errs[i];
            return rcs[i];
        }
    for (int i = 0; i < n; ++i)
        if (rcs[i] == BLOB_RD_ENOTCONV) return BLOB_RD_ENOTCONV;
    return BLOB_RD_OK;
}

// A batch handle: the member handles, their solve kinds, the executor's stream and
// the descriptor tables (in the tail of member 0's workspace).
struct blob_rd_batch {
    std::vector<blob_rd*> hs;
    std::vector<int32_t> kind;
    hipStream_t st = nullptr;
    char* tabs = nullptr;
    size_t tab_bytes = 0;
    int64_t lockstep_max_cells = (int64_t)64 * 64 * 64;
    int32_t threads = 8;
};

int blob_rd_destroy_batch(blob_rd_batch_t b) {
    if (!b) return BLOB_RD_OK;
    for (blob_rd* H : b->hs) blob_rd_destroy(H);
    if (b->st) (void)hipStreamDestroy(b->st);
    delete b;
    return BLOB_RD_OK;
}

int blob_rd_create_batch(const blob_rd_params* p, int32_t n_inst, const int32_t* kind, blob_rd_batch_t* out) {
    if (!out) return g_last_error = "null output handle", BLOB_RD_EINVAL;
    *out = nullptr;
    if (!p || !kind || n_inst <= 0) return g_last_error = "bad argument", BLOB_RD_EINVAL;
    for (int i = 0; i < n_inst; ++i)
        if (kind[i] != 0 && kind[i] != 1) return g_last_error = "kind must be 0 or 1", BLOB_RD_EINVAL;
    const size_t own0 = blob_rd_workspace_bytes(&p[0]);
    if (own0 == 0) return BLOB_RD_EINVAL;
    const size_t tabs = blob_rd_batch_workspace_bytes(n_inst);
    if (!p[0].workspace || p[0].workspace_bytes < own0 + tabs)
        return g_last_error = "member 0's workspace must hold blob_rd_workspace_bytes(&p[0]) + "
                              "blob_rd_batch_workspace_bytes(n_inst) bytes",
               BLOB_RD_ENOMEM;
    blob_rd_batch* b = new blob_rd_batch();
    for (int i = 0; i < n_inst; ++i) {
        blob_rd* H = nullptr;
        const int rc = blob_rd_create(&p[i], &H);
        if (rc != BLOB_RD_OK) {
            g_last_error = "instance " + std::to_string(i) + ": " + g_last_error;
            blob_rd_destroy_batch(b);
            return rc;
        }
        b->hs.push_back(H);
        b->kind.push_back(kind[i]);
        if (kind[i] == 1 && H->P.N <= 0) {
            blob_rd_destroy_batch(b);
            return g_last_error = "absorbing instance " + std::to_string(i) + " has no blobs", BLOB_RD_EINVAL;
        }
    }
    b->tabs = static_cast<char*>(p[0].workspace) + own0;
    b->tab_bytes = p[0].workspace_bytes - own0;
    if (hipStreamCreateWithFlags(&b->st, hipStreamNonBlocking) != hipSuccess) {
        blob_rd_destroy_batch(b);
        return g_last_error = "stream creation failed", BLOB_RD_EDEVICE;
    }
    *out = b;
    return BLOB_RD_OK;
}

blob_rd_t blob_rd_batch_member(blob_rd_batch_t b, int32_t i) {
    if (!b || i < 0 || i >= (int32_t)b->hs.size()) return nullptr;
    return b->hs[i];
}

int blob_rd_batch_set_executor(blob_rd_batch_t b, int64_t lockstep_max_cells, int32_t threads) {
    if (!b || threads < 0) return g_last_error = "bad argument", BLOB_RD_EINVAL;
    b->lockstep_max_cells = lockstep_max_cells;
    b->threads = threads;
    return BLOB_RD_OK;
}

int blob_rd_solve_batch(blob_rd_batch_t b, const double* const* f, double* const* c, double* const* lambda,
                        blob_rd_stats* stats) {
    if (!b || !f || !c) return g_last_error = "null argument", BLOB_RD_EINVAL;
    const int n = (int)b->hs.size();
    return blob_rd_solve_batched(b->hs.data(), n, b->kind.data(), 0.0, f, c, lambda, b->lockstep_max_cells,
                                 b->threads, b->tabs, b->tab_bytes, b->st, stats);
}

}  // extern "C"

// ===========================================================================
// The paper's own solver for the absorbing saddle point (Sec. III.E,
// diffusion-limited case; appendix on preconditioning the saddle-point
// solver): flexible GMRES on the whole block system [A, S; J, 0] with the
// diagonal or the approximate-Schur-complement preconditioner.
extern "C" {

size_t blob_rd_fgmres_workspace_bytes(blob_rd_t H, int restart) {
    if (!H) return 0;
    if (restart <= 0) restart = 30;
    if (restart > kFgMaxRestart) return 0;
    return fg_bytes(H->P, restart);
}

int blob_rd_solve_absorbing_fgmres(blob_rd_t H, double alpha, const blob_rd_saddle_opts* opts, const double* f,
                                   double* c, double* lambda, void* workspace, size_t workspace_bytes,
                                   blob_rd_stats* stt) {
    if (!H || !f || !c || !lambda || !workspace) return g_last_error = "null argument", BLOB_RD_EINVAL;
    if (H->P.N <= 0) return g_last_error = "absorbing solve needs at least one blob", BLOB_RD_EINVAL;
    if (!(alpha >= 0.0) || !std::isfinite(alpha)) return g_last_error = "alpha must be >= 0", BLOB_RD_EINVAL;
    if (reinterpret_cast<uintptr_t>(workspace) % 256) return g_last_error = "workspace not 256-byte aligned",
                                                              BLOB_RD_EINVAL;
    return guarded(H, stt, [&]() {
        const FgOpts o = fg_opts(H, opts);
        if (workspace_bytes < fg_bytes(H->P, o.restart)) throw Err(BLOB_RD_ENOMEM, "FGMRES workspace too small");
        char* ws = static_cast<char*>(workspace);
        int rc = H->P.esz == 4 ? fg_entry<float>(H, alpha, o, f, c, lambda, ws, stt, false)
                               : fg_entry<double>(H, alpha, o, f, c, lambda, ws, stt, false);
        HIPCHK(hipGetLastError());
        return rc;
    });
}

int blob_rd_solve_absorbing_fgmres_noalloc(blob_rd_t H, double alpha, const blob_rd_saddle_opts* opts,
                                           const double* f, double* c, double* lambda, blob_rd_stats* stt) {
    if (!H || !f || !c || !lambda) return g_last_error = "null argument", BLOB_RD_EINVAL;
    if (H->P.N <= 0) return g_last_error = "absorbing solve needs at least one blob", BLOB_RD_EINVAL;
    if (!(alpha >= 0.0) || !std::isfinite(alpha)) return g_last_error = "alpha must be >= 0", BLOB_RD_EINVAL;
    if (!H->noalloc) return g_last_error = "no scratch on this handle's device", BLOB_RD_EDEVICE;
    // a new alpha evicting a cached coarse inverse would also drop captured CG graphs
    bool cached = false;
    for (int k = 0; k < H->cinv_used; ++k) cached = cached || H->cinv_alpha[k] == alpha;
    if (!cached && H->cinv_used == 4) {
        const double old = H->cinv_alpha[H->cinv_next];
        bool captured = false;
        for (const auto& g : H->graphs) captured = captured || g.alpha == old;
        for (const auto& g : H->fg_graphs) captured = captured || g.alpha == old;
        if (captured)
            return g_last_error = "this alpha would evict a captured graph; solve with a cached alpha",
                   BLOB_RD_EINVAL;
    }
    return guarded(H, stt, [&]() {
        const FgOpts o = fg_opts(H, opts);
        const size_t need = fg_bytes(H->P, o.restart);
        if (need > (size_t)BLOB_RD_NOALLOC_BYTES)
            throw Err(BLOB_RD_ENOMEM, "the FGMRES basis needs " + std::to_string(need) + " bytes, more than the " +
                                          std::to_string((size_t)BLOB_RD_NOALLOC_BYTES) +
                                          " of the no-alloc scratch (use a shorter restart or a workspace)");
        std::lock_guard<std::mutex> lk(H->noalloc->use);
        char* ws = H->noalloc->ptr;
        // no graph capture here (instantiating a graph allocates)
        H->fg_capture = false;
        int rc;
        try {
            rc = H->P.esz == 4 ? fg_entry<float>(H, alpha, o, f, c, lambda, ws, stt, false)
                               : fg_entry<double>(H, alpha, o, f, c, lambda, ws, stt, false);
        } catch (...) {
            H->fg_capture = true;
            throw;
        }
        H->fg_capture = true;
        HIPCHK(hipGetLastError());
        HIPCHK(hipStreamSynchronize(H->st));  // the scratch is free again once this returns
        return rc;
    });
}

int blob_rd_schur_apply_cycles(blob_rd_t H, double alpha, const double* x, double* y, int cycles) {
    if (!H || !x || !y || H->P.N <= 0) return g_last_error = "bad argument", BLOB_RD_EINVAL;
    if (!(alpha >= 0.0) || !std::isfinite(alpha) || cycles < 1 || cycles > 64)
        return g_last_error = "bad alpha or cycle count", BLOB_RD_EINVAL;
    return guarded(H, nullptr, [&]() {
        const Plan& P = H->P;
        double* xt = H->nv(2);
        launch_nvec_copy_scale(H->st, x, xt, P.N, 1.0, 0.0);
        if (singular(H, alpha)) launch_nvec_project(H->st, xt, P.N);
        spread_to(H, xt, 0.0, nullptr, H->grid(G_T2), H->inv_h3(), nullptr);
        const double* cinv = select_cinv(H, alpha);
        if (P.esz == 4) fg_cycles<float>(H, alpha, H->grid(G_T2), nullptr, 0.0, H->grid(G_U), true, cycles, cinv);
        else fg_cycles<double>(H, alpha, H->grid(G_T2), nullptr, 0.0, H->grid(G_U), true, cycles, cinv);
        fg_interp(H, H->grid(G_U), y);
        if (singular(H, alpha)) launch_nvec_project(H->st, y, P.N);
        HIPCHK(hipGetLastError());
        HIPCHK(hipStreamSynchronize(H->st));
        return BLOB_RD_OK;
    });
}

int blob_rd_saddle_precond(blob_rd_t H, double alpha, const blob_rd_saddle_opts* opts, const double* vg,
                           const double* vf, double* zg, double* zl) {
    if (!H || !vg || !vf || !zg || !zl) return g_last_error = "null argument", BLOB_RD_EINVAL;
    if (H->P.N <= 0) return g_last_error = "the saddle preconditioner needs at least one blob", BLOB_RD_EINVAL;
    if (!(alpha >= 0.0) || !std::isfinite(alpha)) return g_last_error = "alpha must be >= 0", BLOB_RD_EINVAL;
    return guarded(H, nullptr, [&]() {
        const FgOpts o = fg_opts(H, opts);
        if (H->P.esz == 4) fg_precond<float>(H, alpha, o, vg, vf, zg, zl);
        else fg_precond<double>(H, alpha, o, vg, vf, zg, zl);
        HIPCHK(hipGetLastError());
        HIPCHK(hipStreamSynchronize(H->st));
        return BLOB_RD_OK;
    });
}

}  // extern "C"
