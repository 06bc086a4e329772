// Host-side launchers for the blob_rd kernels (all enqueue on `st`).
#pragma once

#include "brd.hpp"

namespace brd {

// ---- natural-layout FP64 grid kernels ------------------------------------
// q = alpha p - D L p ; partials (p.q, sum q) into part[0..1][nb]
void launch_applyA(hipStream_t st, const double* p, double* q, double alpha, double s, int nx, int ny,
                   int nz, double* part, const Scalars* sc, unsigned* nparts_out);
// y = alpha x - D L x (no partials, no guard); box: L with homogeneous box faces
void launch_applyA_plain(hipStream_t st, const double* x, double* y, double alpha, double s, int nx, int ny,
                         int nz, bool box = false);
// q = base - (alpha x - D L x) in one pass (box: homogeneous box faces); q must not alias x
void launch_residA_plain(hipStream_t st, const double* base, const double* x, double* q, double alpha, double s,
                         int nx, int ny, int nz, bool box = false);
// partials (g.g, sum g, g.g) of a residual that already holds g
void launch_self_partials(hipStream_t st, const double* g, size_t n, double* part, unsigned* nparts_out);
// r = g - q0 (q0 may be null: r = g); partials (r.r, sum r, g.g)
void launch_residual_from_q(hipStream_t st, const double* g, const double* q0, double* r, size_t n, double* part,
                            unsigned* nparts_out);
// Two-cells-per-thread forms (nx even): stencil with partials, direction update,
// CG update, z dots.
void launch_applyA2(hipStream_t st, const double* p, double* q, double alpha, double s, int nx, int ny, int nz,
                    double* part, const Scalars* sc, unsigned* nparts_out, bool box = false);
// p = z + shift + beta p (z split, level-0 layout of type T)
template <typename T>
void launch_dir2(hipStream_t st, const T* z0, const T* z1, double* p, int nx, int ny, int nz, const Scalars* sc);
// x += alpha p ; r -= alpha q with partials (r.r, sum r), and the V-cycle entry of
// the new r (f split, first red sweep u0); box_inv: per-face-count inverse
// diagonals of a box with fixed faces (inv_diag unused)
template <typename T>
void launch_update2_enter(hipStream_t st, double* x, double* r, const double* p, const double* q, T* f0, T* f1, T* u0,
                          int nx, int ny, int nz, double inv_diag, double* part, const Scalars* sc,
                          unsigned* nparts_out, const BoxCoef* box_inv = nullptr);
// partials (sum z, z.r, z.q) with z split of type T
template <typename T>
void launch_zdots2(hipStream_t st, const T* z0, const T* z1, const double* r, const double* q, int nx, int ny, int nz,
                   double* part, const Scalars* sc, unsigned* nparts_out);
// out = scale * out + z (+ shift_scale * *shift_dev): z split -> natural FP64
template <typename T>
void launch_split_to_nat(hipStream_t st, const T* z0, const T* z1, double* out, int nx, int ny, int nz,
                         double scale_in_place, const double* shift_dev = nullptr, double shift_scale = 0.0);
// out = (b + z) + shift_scale * *shift_dev (b, z split; nx even)
template <typename T>
void launch_split_add_to_nat(hipStream_t st, const T* b0, const T* b1, const T* z0, const T* z1, double* out, int nx,
                             int ny, int nz, const double* shift_dev, double shift_scale);
// sums (sum v, v.v) of a natural vector
void launch_norm_partials(hipStream_t st, const double* v, size_t n, double* part, unsigned* nparts_out);
void launch_fill(hipStream_t st, double* v, size_t n, double value);
void launch_axpby(hipStream_t st, double* y, const double* x, size_t n, double a, double b);  // y = a y + b x
void launch_add_shift(hipStream_t st, double* v, size_t n, const double* shift_dev, double sign);

// ---- long [grid; blobs] vectors of the flexible GMRES on the saddle system ----
// w -= (*hprev) vprev (if vprev), partials of w.vnext (w.w if vnext is null)
void launch_fg_mgs(hipStream_t st, double* w, const double* vprev, const double* hprev, const double* vnext,
                   size_t n, double* part, unsigned* np);
// Classical Gram-Schmidt for the flexible GMRES basis (v_k = V + k * stride, k < m):
// out[k] = w . v_k (groups of `group` <= 8 vectors per pass over w; *wn2 = w.w when wn2 is set),
// then w -= sum_k h[k] v_k with *hout = |w|; the first update (add null) sets *redo when
// |w|^2 < eta2 * *pre2, a second one (gate = redo) adds `add` into col. A set gate reading 0
// makes every launch a no-op. part needs (group + 1) * fg_cgs_blocks(n) doubles.
unsigned fg_cgs_blocks(size_t n);
void launch_fg_cgs_dots(hipStream_t st, const double* w, const double* V, size_t stride, size_t n, int m, int group,
                        double* out, double* wn2, double* part, const int* gate);
void launch_fg_cgs_update(hipStream_t st, double* w, const double* V, size_t stride, size_t n, const double* h, int m,
                          double* part, const int* gate, double* hout, const double* pre2, double eta2, int* redo,
                          double* col, const double* add);
// *out = sum of partials (sqrt of it with take_sqrt)
void launch_fg_fin(hipStream_t st, const double* part, unsigned np, double* out, int take_sqrt);
// w /= *h (0 if *h == 0)
void launch_fg_scale(hipStream_t st, double* w, const double* h, size_t n);
void launch_fg_scale_sum(hipStream_t st, double* w, const double* h, size_t n, size_t ncell, double* part,
                         unsigned* np);
// r = [bg; phi] - r (sub) or [bg; phi] (phi a constant on every blob); partials of r.r
void launch_fg_resid(hipStream_t st, double* r, const double* bg, size_t ncell, size_t n, int sub, double* part,
                     unsigned* np, double phi = 0.0);
// x[0..n) += sum_j y_j Z_j[off ..) (y on the device)
void launch_fg_update(hipStream_t st, double* x, const double* Z, size_t stride, size_t off, size_t n, int k,
                      const double* y);
// Hessenberg column j (column-major, leading dimension ld): rotations, residual
// estimate out[0] = |g[j+1]|, out[1] = subdiagonal before rotation
void launch_fg_givens(hipStream_t st, double* Hd, int ld, double* cs, double* sn, double* g, int j, double* out);
void launch_fg_gstart(hipStream_t st, double* g, int len, const double* beta);
void launch_fg_backsolve(hipStream_t st, const double* Hd, int ld, const double* g, double* y, int k);

// ---- finalize kernels (one work-group) ------------------------------------
enum FinKind { FIN_INIT = 0, FIN_ALPHA = 1, FIN_UPDATE = 2, FIN_BETA = 3 };
void launch_fin(hipStream_t st, int kind, const double* part, unsigned nparts, Scalars* sc,
                const double* nvec_a, const double* nvec_b, int nblob, double inv_h3);
// sum of partial sets into out[0..k-1] (generic)
void launch_reduce_parts(hipStream_t st, const double* part, unsigned nparts, int k, double* out);

// ---- multigrid (split layout) ---------------------------------------------
template <typename T>
void launch_enter(hipStream_t st, const double* r, T* f0, T* f1, T* u0, int nx, int ny, int nz,
                  double inv_diag, const Scalars* sc);
// entry from the residual g - A c of a split-layout guess c (periodic, nx even; u0 may be null)
template <typename T>
void launch_resid_enter(hipStream_t st, const double* g, const T* c0, const T* c1, T* f0, T* f1, T* u0, int nx,
                        int ny, int nz, double alpha, double s, double inv_diag);
template <typename T>
void launch_gs(hipStream_t st, T* uc, const T* uo, const T* fc, int hx, int ny, int nz, int color, double s,
               double inv_diag, const Scalars* sc, int bs = kBlock);
// the first half-sweep of colour `color` after a V-cycle entry, reading the other colour's f
// fo and scaling it by inv_diag (the entry's zero-guess sweep) instead of its u; returns false
// (nothing launched) when the rows do not take the vector form
template <typename T>
bool launch_gs_from_f(hipStream_t st, T* uc, const T* fo, const T* fc, int hx, int ny, int nz, int color, double s,
                      double inv_diag, const Scalars* sc, int bs = kBlock);
// closing red half-sweep of the finest level + partials (sum z, z.r, z.q); returns
// the partial count, 0 if not applicable (nothing launched)
template <typename T>
unsigned launch_gs_dots(hipStream_t st, T* uc, const T* uo, const T* fc, int hx, int ny, int nz, double s,
                        double inv_diag, const double* r, const double* q, double* part, const Scalars* sc,
                        int bs = kBlock);
// red residual after pre-smoothing (the black one is zero after the closing black half-sweep)
template <typename T>
void launch_resid_red(hipStream_t st, const T* u0, const T* u1, const T* f0, T* r0, int hx, int ny, int nz, double s,
                      double diag, const Scalars* sc, int bs = kBlock);
// fine red residual -> coarse f (split, with zero-guess red update) or natural (coarsest)
template <typename T>
void launch_restrict(hipStream_t st, const T* r0, int nx, int ny, int nz, T* cf0, T* cf1, T* cu0, int coarse_natural,
                     double inv_diag_c, const Scalars* sc, int bs = kBlock);
template <typename T>
void launch_prolong(hipStream_t st, const T* cu0, const T* cu1, int coarse_natural, T* u0, T* u1, int nx, int ny,
                    int nz, const Scalars* sc, int bs = kBlock);
template <typename T>
void launch_coarse(hipStream_t st, const T* f, T* u, const double* cinv, int m, const Scalars* sc);

// ---- multigrid of a box with homogeneous faces (split layout, one cell per thread) ----
// The same V-cycle steps as above with the box operator: per-cell diagonals from
// the face count (BoxCoef, index = faces touched), no neighbours across faces,
// restriction and prolongation with the ghost -u beyond a face.
template <typename T>
void launch_enter_box(hipStream_t st, const double* r, T* f0, T* f1, T* u0, int nx, int ny, int nz,
                      const BoxCoef& inv, const Scalars* sc);
template <typename T>
void launch_gs_box(hipStream_t st, T* uc, const T* uo, const T* fc, int nx, int ny, int nz, int color, double s,
                   const BoxCoef& inv, const Scalars* sc);
template <typename T>
void launch_resid_red_box(hipStream_t st, const T* u0, const T* u1, const T* f0, T* r0, int nx, int ny, int nz,
                          double s, const BoxCoef& diag, const Scalars* sc);
template <typename T>
void launch_restrict_box(hipStream_t st, const T* r0, int nx, int ny, int nz, T* cf0, T* cf1, T* cu0,
                         int coarse_natural, const BoxCoef& inv_c, const Scalars* sc);
template <typename T>
void launch_prolong_red_box(hipStream_t st, const T* cu0, const T* cu1, int coarse_natural, T* u0, int nx, int ny,
                            int nz, const Scalars* sc);
// the box V-cycle below level t in one work-group (levels in LDS), as launch_tail
template <typename T>
void launch_tail_box(hipStream_t st, const T* f0, const T* f1, T* u0, T* u1, const TailDesc& d, const double* cinv,
                     const Scalars* sc);
template <typename T>
hipError_t tail_box_set_lds(size_t bytes);

template <typename T>
void launch_tail(hipStream_t st, const T* f0, const T* f1, T* u0, T* u1, const TailDesc& d, const double* cinv,
                 const Scalars* sc);
template <typename T>
hipError_t tail_set_lds(size_t bytes);
// temporally blocked level (nx, ny, nz divisible by 8): pre-smoothing + red residual +
// restriction (pre-smoothed red to ured); red correction + post-smoothing from ured
template <typename T>
void launch_down(hipStream_t st, const T* u0, const T* f0, const T* f1, T* ured, int nx, int ny, int nz, double s,
                 double diag, T* cf0, T* cf1, T* cu0, double inv_diag_c, const Scalars* sc);
template <typename T>
void launch_up(hipStream_t st, const T* cu0, const T* cu1, const T* ured, const T* f0, const T* f1, T* u0, T* u1,
               int nx, int ny, int nz, double s, double diag, const Scalars* sc);
template <typename T>
hipError_t blocked_set_lds();

// ---- batched launches (one launch per step for every instance of a batch) ----
enum { BCG_DIR = 0, BCG_APPLY, BCG_UPDATE, BCG_FIN_ALPHA, BCG_FIN_UPDATE, BCG_FIN_BETA };
enum { BMG_GS = 0, BMG_GS_DOTS, BMG_RESID, BMG_RESTRICT, BMG_PROLONG, BMG_TAIL };
// CG steps over the work list `tab` with a fixed grid of `grid` work-groups;
// the fin kinds take one work-group per instance (ninst)
template <typename T>
void launchb_cg(hipStream_t st, int what, const InstDev* inst, const int* gate, const BatchTab* tab, unsigned grid,
                int ninst);
// V-cycle steps on level l; BMG_TAIL takes one work-group per instance (grid = ninst) with lds bytes
template <typename T>
void launchb_mg(hipStream_t st, int what, const InstDev* inst, const int* gate, const BatchTab* tab, unsigned grid,
                int l, int color, unsigned lds);
template <typename T>
hipError_t tail_set_lds_batched(size_t bytes);
// measurement probe: out = a + b over `bytes` bytes of 16-byte vectors
void launch_stream_add(hipStream_t st, const void* a, const void* b, void* out, size_t bytes);
// blob term: interp (spread = 0) or spread (1)
void launchb_blob(hipStream_t st, int spread, const InstDev* inst, const int* gate, const BatchTab* tab,
                  unsigned grid);

// ---- blobs -----------------------------------------------------------------
// wrap positions, kernel weights, tile ids, bin counts (int atomics on counts only)
void launch_blob_setup(hipStream_t st, const double* q, int N, BlobGeom g, int* base /*[3N]*/,
                       double* wts /*[12N]*/, int* tile_of, int* counts);
void launch_bin_scan(hipStream_t st, const int* counts, int ntiles, int* offsets /*ntiles+1*/);
void launch_bin_scatter(hipStream_t st, const int* tile_of, int N, const int* offsets, int* cursor, int* perm);
void launch_bin_sort(hipStream_t st, const int* offsets, int ntiles, int* perm);
// out[i] = scale_i * (J x)_i, scale = kappa (if non-null) ; jx (optional) gets (J x)_i
void launch_interp(hipStream_t st, const double* x, int N, BlobGeom g, const int* base, const double* wts,
                   const int* perm, double* jx, const double* kappa, double* out, const Scalars* sc);
// out_i = (J z)_i for z held in a red/black split level-0 layout (z0, z1 of type T)
template <typename T>
void launch_interp_split(hipStream_t st, const T* z0, const T* z1, int N, BlobGeom g, const int* base,
                         const double* wts, const int* perm, double* out);

// contribution lists of the spread (mode 0: per-tile counts into cnt[0..2 ntiles);
// mode 1: lists at the scanned offsets offE, offC)
void launch_spread_plan(hipStream_t st, int mode, BlobGeom g, const int* base, const double* wts, const int* offsets,
                        const int* perm, int* cnt, const int* offE, const int* offC, int* tcell, int* tptr,
                        int* tblob, double* tw);
// out[c] = base(c) + scale * sum_e w m(blob) over the touched cells only
void launch_spread_sparse(hipStream_t st, const SpreadLists& L, const SpreadMult& M, const double* base_in,
                          double* out, double scale, const Scalars* sc);
// V-cycle entry of r = base + scale S m at the touched cells (split f, u_red = f_red / diag);
// u0, and f0/f1 elsewhere, must already hold zeros (no base) or k_enter's values of base_in.
// u0 null: u_red is not written (a cycle that opens from f)
template <typename T>
void launch_spread_enter(hipStream_t st, const SpreadLists& L, const SpreadMult& M, const double* base_in,
                         double scale, T* f0, T* f1, T* u0, int nx, int ny, double inv_diag);
// the same entry at a spread term's touched cells: (g - A c) + scale S m (after launch_resid_enter)
template <typename T>
void launch_resid_spread_enter(hipStream_t st, const SpreadLists& L, const SpreadMult& M, const double* g,
                               const T* c0, const T* c1, double scale, T* f0, T* f1, T* u0, int nx, int ny, int nz,
                               double alpha, double s, double inv_diag);
template <typename T>
void launch_zero(hipStream_t st, T* p, size_t n);
template <typename T>
void launch_copy2(hipStream_t st, const T* a0, const T* a1, T* b0, T* b1, size_t n);

// ---- N-vector kernels (single work-group) ------------------------------------
void launch_nvec_project(hipStream_t st, double* v, int N);  // v -= mean(v)
// Fourier coarse level of the Schur preconditioner (columns stored one after another)
void launch_coarse_basis(hipStream_t st, const double* q, int N, const int* mv, int nmodes, double kx, double ky,
                         double kz, double* Z);
void launch_coarse_gram(hipStream_t st, const double* Z, const double* Y, int N, int K, double* E);
int coarse_chunks(int N);  // row chunks of the coarse-level dot products
// with_sum: also the chunk sums of v (column K of part, which then needs K + 1 columns)
void launch_coarse_dots(hipStream_t st, const double* A, int N, int K, const double* v, double* part,
                        bool with_sum = false);
// sub_mean: out = (x - mean x) + Y c, the mean from column K of part
void launch_coarse_update(hipStream_t st, const double* part, const double* base, int K, double sgn, const double* Y,
                          int N, const double* x, double* out, double* a_out, bool sub_mean = false);
void launch_coarse_rotate(hipStream_t st, const double* Y, const double* Einv, int N, int K, double* out);
void launch_nvec_copy_scale(hipStream_t st, const double* x, double* y, int N, double a, double shift);
// v_0 = r / |r|, r = b - w (has_w) or b with its mean removed when project is set; g_0 = |r|
void launch_gmres_start(hipStream_t st, const double* b, const double* w, int has_w, double* V, double* g, int N,
                        GmresScalars* gs, int project = 0);
// Arnoldi step k (V_{k+1} holds the product; project: remove its mean first)
void launch_gmres_arnoldi(hipStream_t st, double* V, double* H, double* cs, double* sn, double* g, int N, int k,
                          int m, GmresScalars* gs, int project = 0);
void launch_gmres_update(hipStream_t st, const double* V, const double* H, const double* g, double* y, double* x,
                         int N, int k, int m);
void launch_nvec_sums(hipStream_t st, const double* a, const double* b, int N, double* out /*sum a, a.a, a.b*/);

// ---- learned preconditioner -------------------------------------------------
void launch_pair_cells(hipStream_t st, const double* q, int N, PairGeom pg, int* cell_of, int* counts);
void launch_pair_count(hipStream_t st, const double* q, int N, PairGeom pg, const int* cell_of, const int* offsets,
                       const int* perm, int* cnt);
void launch_pair_fill(hipStream_t st, const double* q, int N, PairGeom pg, const int* cell_of, const int* offsets,
                      const int* perm, const int* rowptr, int* col, int* rowidx);
void launch_rowidx(hipStream_t st, const int* rowptr, int N, int* rowidx);
void launch_pair_nu(hipStream_t st, const double* q, PairGeom pg, const int* rowptr, const int* col, int N, float* nu);
void launch_net_assemble(hipStream_t st, const double* q, PairGeom pg, NetDev net, const int* col, const int* rowidx,
                         long long nnz, double Dh, double diag, double* val);
void launch_spmv(hipStream_t st, const int* rowptr, const int* col, const double* val, const double* x, double* y,
                 int N);
// y = W (x - mean(x))
void launch_spmv_centered(hipStream_t st, const int* rowptr, const int* col, const double* val, const double* x,
                          double* y, int N);
void launch_count_bad(hipStream_t st, const double* v, long long n, int* out);
void launch_entry_grad(hipStream_t st, const int* rowidx, const int* col, long long nnz, const double* RP,
                       const double* YP, const double* coef, int S, int N, double half_Dh, float* dg);
int launch_net_backward(hipStream_t st, const double* q, PairGeom pg, NetDev net, const int* col, const int* rowidx,
                        long long nnz, const float* dg, float* wpart, int max_waves);
void launch_grad_reduce(hipStream_t st, const float* wpart, int nwaves, float* grad);
void launch_adam(hipStream_t st, float* P, float* m, float* v, const float* grad, float lr, float b1, float b2,
                 float eps, int t);
void launch_net_pack(hipStream_t st, const float* P, __bf16* W1b, __bf16* W2b, __bf16* w3b);

}  // namespace brd
