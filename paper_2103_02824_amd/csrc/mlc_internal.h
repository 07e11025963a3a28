// Internal state of an mlc context (host side) and the launch interface of the
// gfx950 kernels. Not part of the ABI.
#pragma once

#include <cstdint>
#include <string>
#include <vector>

#include <hip/hip_runtime.h>

#include "../../include/mlc.h"
#include "chunks.h"
#include "p2.h"

namespace mlc {

// Symmetric 4-point quadrature of degree 2 on a tetrahedron: barycentric
// points (a,b,b,b) and permutations, weight |T|/4 each.
constexpr double QA = 0.58541019662496845446;  // (5 + 3 sqrt 5) / 20
constexpr double QB = 0.13819660112501051518;  // (5 - sqrt 5) / 20

// Device sub-buffers carved out of the caller's workspace.
struct Dev {
  // fine mesh (library orders)
  int32_t* tets = nullptr;      // nt x ne fine node ids (ne = 4 for P1, 10 for P2)
  int32_t* v2d = nullptr;       // nv: vertex -> dof or -1
  double* xyz = nullptr;        // nv x 3
  double* geo = nullptr;        // nt x 16: vol, grad lambda_0..3 (12), pad
  double* qpx = nullptr;        // nt x nq x 3 quadrature point coordinates (fields below: nt x nq)
  double* qtab = nullptr;       // P2 reference tables (p2.h), order 2 only
  double* vext = nullptr;       // nt x 4
  double* vxc = nullptr;        // nt x 4   V_xc(rho^l)
  double* exc = nullptr;        // nt x 4
  double* veff = nullptr;       // nt x 4
  double* rho = nullptr;        // nt x 4   rho^l
  double* fld = nullptr;        // nt x 4   V_ext + V_xc + g
  double* fld2 = nullptr;       // nt x 4   w0
  double* rhot = nullptr;       // nt x 4   density of normalised u_i
  int32_t* rowptr = nullptr;    // n + 1
  int32_t* col = nullptr;       // nnz
  int32_t* adj_ptr = nullptr;   // n + 1
  int32_t* adj_tet = nullptr;   // nadj
  int8_t* adj_loc = nullptr;    // nadj
  int32_t* bverts = nullptr;    // boundary vertex ids
  // operators on the interior CSR pattern
  double* valA = nullptr;       // A + sigma M (step 5)
  double* valF = nullptr;       // A_fix = 1/2 K + M_{V_ext + V_xc + g}
  double* valW = nullptr;       // M_{w0}
  double* valM = nullptr;       // M
  double* valK = nullptr;       // K
  double* elem = nullptr;       // element entries of two operators in slot order (2 ns; also load scratch)
  int32_t* slot_ptr = nullptr;  // nnz + 1
  int32_t* slot_of = nullptr;   // nt x 16: slot-order position of element entry (a, b)
  int32_t* diag_slot = nullptr; // n
  double* dinvA = nullptr;      // n
  double* dinvK = nullptr;      // n
  // orbital blocks, n x N row-major
  double* Phi = nullptr;        // Phi^l (state)
  double* X = nullptr;          // CG iterate, then u_i
  double* R = nullptr;
  double* P = nullptr;
  double* Q = nullptr;
  double* B = nullptr;
  double* Y = nullptr;          // 4 blocks of n x N
  double* Yh = nullptr;         // Hartree solver scratch, 4 n (polynomial Z0, Z1, d; coarse-corrected z)
  double* red2 = nullptr;       // partials of the Gram blocks computed beside the Hartree solve
  // single vectors
  double* w = nullptr;          // nv nodal Hartree potential
  double* g = nullptr;          // nv multipole data (0 inside)
  double* w0 = nullptr;         // n
  double* lvec = nullptr;       // n   l = K_IB g_B
  double* pb = nullptr;         // n
  double* pr = nullptr;         // n
  double* pp = nullptr;         // n
  double* pq = nullptr;         // n
  double* rho_nodal = nullptr;  // nv
  // prolongation
  int32_t* Pk = nullptr;        // n x 4
  double* Pw = nullptr;         // n x 4
  // chunked restriction P^T Y: fine rows in chunks of RCH; per chunk the
  // (local row, weight) entries grouped by coarse DoF into segments; per coarse
  // DoF its segments in chunk order; partial sums per segment (nseg x N)
  int32_t* rch_seg = nullptr;   // nchunk + 1
  int32_t* rseg_ptr = nullptr;  // nseg + 1
  int32_t* rent_row = nullptr;  // nent
  double* rent_w = nullptr;     // nent
  int32_t* kseg_ptr = nullptr;  // nH + 1
  int32_t* kseg = nullptr;      // nseg
  double* rpart = nullptr;      // nseg x N
  double* rpartH = nullptr;     // nseg: the Hartree CG's coarse correction (beside the Gram blocks)
  int32_t* PTptr = nullptr;     // nH + 1
  int32_t* PTidx = nullptr;
  double* PTw = nullptr;
  // coarse grouping
  int32_t* cgrp_ptr = nullptr;  // cnt + 1
  int32_t* cgrp_tet = nullptr;  // nt
  int32_t* cgrp_dof = nullptr;  // 4 nt: DoFs of the fine tets in coarse-group order (-1: boundary)
  double* cgeo = nullptr;       // cnt x 12
  double* cel_ops = nullptr;    // cnt x 40
  double* cel_orb = nullptr;    // cnt x N x 14
  double* cel_tri = nullptr;    // cnt x 20
  double* cel_pairs = nullptr;  // joint variant: cnt x npair x 4, (u_j u_l, psi_m)
  int32_t* pair_jl = nullptr;   // joint variant: the pairs (j <= l), 2 x npair
  int32_t* nbr = nullptr;       // estimator: nt x 4, tet across the face opposite vertex a (-1: boundary)
  int32_t* tord = nullptr;      // estimator: the caller's index of each (Morton-ordered) tet
  double* chat = nullptr;       // 17 x nt: coarse hats at fine quadrature points, fine volume
  // small
  double* small = nullptr;      // packed small blocks (see step.cpp)
  double* coarse_in = nullptr;  // phi_H (nH x N), w_H (nH), theta2 (N)
  double* occ = nullptr;        // N
  double* RZ = nullptr;         // 4 x n_nuclei
  double* colv = nullptr;       // 2 x N per-column scratch
  double* red = nullptr;        // reduction partials
  double* scal = nullptr;       // 2 x 5N CG scalars (orbitals), two parity buffers
  double* scalP = nullptr;      // 2 x 5 CG scalars (Hartree)
  int32_t* flags = nullptr;     // [0] active (buffer 0) [2] active (buffer 1) [4] breakdown
  int32_t* flagsP = nullptr;
  // FP32 inner solve of the iterative refinement
  float* valA32 = nullptr;      // nnz
  float* dinvA32 = nullptr;     // n
  float *X32 = nullptr, *R32 = nullptr, *P32 = nullptr, *Q32 = nullptr, *B32 = nullptr;  // n x N
  double* scal32 = nullptr;     // 2 x 5N
  int32_t* flags32 = nullptr;   // 8
  // learned initial guess of step 5
  float* F = nullptr;           // n N x 6 features (row i N + c)
  float* Ynn = nullptr;         // n N network outputs
  double* gscale = nullptr;     // N: max |phi_c|
  double* gsel = nullptr;       // 4N: [learned start used, |r|^2 span minimiser, |r|^2 plain, |r|^2 taken]
  double* gdots = nullptr;      // 5N: Galerkin sums of the learned start
  int32_t* d2v = nullptr;       // n: library dof -> vertex
  int32_t* dof_user = nullptr;  // n: library dof -> caller dof
  int32_t* chk = nullptr;       // 4: count of non-finite inputs (mlc_set_state)
  double* lmax = nullptr;       // 2: upper ends of the Chebyshev intervals of D^-1 A (step 5) and D^-1 K (Hartree)
  double* lanc = nullptr;       // 2 x 64 + 4: Lanczos coefficients of the lmax estimate
  float* valK32 = nullptr;      // nnz: K in FP32 for the Hartree CG's polynomial steps
  double* KHinv = nullptr;      // nH x nH: inverse of the coarse stiffness (two-level Hartree CG)
  double* rH = nullptr;         // nH: restricted residual
  double* eH = nullptr;         // nH: coarse correction
};

struct Options {
  mlc_options o;
};

}  // namespace mlc

struct mlc_ctx {
  // ---- inputs -------------------------------------------------------------
  int64_t nv = 0, nt = 0, cnv = 0, cnt = 0;   // nv: fine nodes (P1: the vertices)
  int32_t order = 1, ne = 4, nq = 4;    // element order, nodes and quadrature points per fine tet
  int64_t nvert = 0;                    // fine vertices (the first nvert nodes)
  std::vector<double> qtab;             // P2 reference tables (order 2)
  std::vector<double> xyz, cxyz;        // fine nodes in caller order (vertices, then P2 edge midpoints)
  std::vector<int32_t> tets;            // nt x ne node ids, library tet order (Morton by centroid)
  std::vector<int32_t> ctets;
  int32_t n_nuclei = 0;
  std::vector<double> R, Z, occ;
  int32_t potential = 0, xc = 0, hartree = 1, N = 1;
  double rc = 0.5, omega = 1.0, xalpha = 0.77298;
  double lo[3] = {0, 0, 0}, hi[3] = {0, 0, 0};  // the box, per axis
  mlc_options opt{};
  // ---- fine DoFs ----------------------------------------------------------
  int64_t n = 0;                        // interior DoFs
  std::vector<int32_t> v2d, d2v;        // vertex <-> library dof
  std::vector<int32_t> dof_user;        // library dof -> caller dof index
  std::vector<int32_t> bverts;
  std::vector<int32_t> rowptr, col;
  std::vector<int32_t> adj_ptr, adj_tet;
  std::vector<int8_t> adj_loc;
  std::vector<double> geo;              // nt x 16
  std::vector<int32_t> tord;            // caller's index of each library tet (estimator option)
  std::vector<int32_t> nbr;             // nt x 4 face neighbours (estimator option)
  std::vector<int32_t> slot_ptr, slot_of, diag_slot;  // assembly lists
  // ---- coarse ---------------------------------------------------------------
  int64_t nH = 0;
  std::vector<int32_t> cv2d, cd2v;
  std::vector<int32_t> Pk;              // n x 4
  std::vector<double> Pw;
  std::vector<int32_t> PTptr, PTidx;
  std::vector<double> PTw;
  std::vector<int32_t> rch_seg, rseg_ptr, rent_row, kseg_ptr, kseg;  // chunked restriction (see Dev)
  std::vector<double> rent_w;
  std::vector<int32_t> parent;          // fine tet -> coarse tet
  std::vector<int32_t> cgrp_ptr, cgrp_tet, cgrp_dof;
  std::vector<double> cgeo;             // cnt x 12
  std::vector<double> cvol;             // coarse tet volumes
  std::vector<double> Pfull_w;          // nv x 4 weights (all fine vertices, coarse vertex ids)
  std::vector<int32_t> Pfull_k;
  // ---- device ---------------------------------------------------------------
  char* ws = nullptr;
  size_t ws_bytes = 0;
  hipStream_t stream = nullptr;
  mlc::Dev d;
  bool bound = false, has_state = false, has_step = false;
  int64_t nred = 0;                     // size of reduction partial buffer (doubles)
  // ---- state ----------------------------------------------------------------
  std::vector<double> lam;
  // host copies of the last step's small blocks (for mlc_probe and the inner loop)
  std::vector<double> h_tri;            // cnt x 20 (once per mesh)
  std::vector<double> h_Mh_chol;        // dense L of M_H (once per mesh)
  std::vector<double> h_KH;             // dense C_H = P^T K P (once per mesh)
  std::vector<double> h_Kh_chol;        // its Cholesky factor
  std::vector<double> h_MH;             // dense M_H
  std::vector<double> h_KHinv;          // K_H^-1 (two-level Hartree CG; once per mesh)
  std::vector<double> last_theta2, last_phiH, last_wH;
  double last_theta1 = 0.0, last_sigma = 0.0;
  std::vector<double> last_small;       // packed small blocks of the fine stage
  std::vector<double> last_cel_ops, last_cel_orb, last_cel_pairs;
  int64_t small_len = 0;
  std::string err;
  // timing of the dominant kernel
  std::vector<hipEvent_t> ev_pool;
  int ev_used = 0;
  // captured CG iteration chunks per solve kind (0 orbitals, 1 Hartree, 2
  // orbitals FP32) and size (2 << g iterations), the tolerance and
  // preconditioner they were captured with, and the last solve's iterations
  hipGraphExec_t cg_graph[3][mlc::CHUNK_GRAPHS] = {};
  double cg_graph_rt2[3] = {0.0, 0.0, 0.0};
  int cg_graph_pc[3] = {0, 0, 0};      // polynomial degree + 100 with the coarse correction (0: Jacobi)
  int cg_pred[3] = {0, 0, 0};
  hipStream_t cap_stream = nullptr;     // library-owned stream used only to record graphs
  hipStream_t side = nullptr;           // library-owned stream for work beside the Hartree solve
  hipEvent_t ev_fork = nullptr, ev_join = nullptr;
  // learned initial guess of step 5 and the sample sink that feeds its training
  const mlc_nn* nn = nullptr;
  float* sink_x = nullptr;
  float* sink_t = nullptr;
  int64_t sink_cap = 0, sink_count = 0;
  int32_t sink_stride = 1;
};

namespace mlc {

struct NnDev;
const NnDev* nn_device(const mlc_nn* nn);

// ---- host helpers -----------------------------------------------------------
mlc_status fail(mlc_ctx* c, mlc_status s, const std::string& msg);
mlc_status hip_fail(mlc_ctx* c, hipError_t e, const char* what);

mlc_status build_mesh(mlc_ctx* c, const mlc_mesh* fine, const mlc_mesh* coarse);
size_t workspace_layout(mlc_ctx* c, char* base, Dev* d);
mlc_status upload_and_init(mlc_ctx* c);
mlc_status fine_stage_and_step(mlc_ctx* c, mlc_step_report* rep);
mlc_status coarse_scf(mlc_ctx* c, double tol, int maxit, int* iters);
mlc_status probe(mlc_ctx* c, int which, double* out, int64_t count);

// ---- kernel launchers (kernels.hip) -------------------------------------------
int spmm_rows_per_block(int N);

// Chebyshev polynomial preconditioner of one CG solve (null pointer: Jacobi).
// Preconditioner of the Hartree CG: hartree_precond, or precond when it is -1.
inline int hartree_pc(const mlc_options& o) { return o.hartree_precond < 0 ? o.precond : o.hartree_precond; }
inline int hartree_deg(const mlc_options& o) { return o.hartree_cheb_degree > 0 ? o.hartree_cheb_degree : o.cheb_degree; }
inline double hartree_ratio(const mlc_options& o) { return o.hartree_cheb_ratio > 0 ? o.hartree_cheb_ratio : o.cheb_ratio; }

template <typename T>
struct PolyPC {
  const double* lmax;  // device scalar: Gershgorin bound of D^-1 A
  double ratio;        // interval [lmax / ratio, lmax]
  int degree;          // >= 2
  T* Z[2];             // ping-pong blocks of the iterates, n x N each
  double* rz_part;     // per-block r.z partials of the last step (spmm_blocks(n, N) x N)
  const float* val32 = nullptr;  // optional FP32 copy of the matrix values for the steps (FP64, one column)
};
template <typename T>
void launch_cg_init_t(hipStream_t s, int64_t n, int N, const T* B, const T* AX, const T* dinv, T* Rv, T* P,
                      double* partial, const PolyPC<T>* pc);
template <typename T>
void launch_cg_update_t(hipStream_t s, int64_t n, int N, const T* dinv, T* X, T* Rv, const T* P, const T* Q,
                        const double* pq_part, const double* scal, const int32_t* flags, double* partial,
                        int32_t* brk, const PolyPC<T>* pc);
template <typename T>
void launch_cg_direction_t(hipStream_t s, int64_t n, int N, const T* dinv, const T* Rv, T* P, const double* upd_part,
                           const double* scal_in, const int32_t* flags_in, double* scal_out, int32_t* flags_out,
                           double rtol2, const PolyPC<T>* pc);
template <typename T>
void launch_cheb_steps_t(hipStream_t s, int64_t n, int N, const int32_t* rowptr, const int32_t* col, const T* val,
                         const T* dinv, const T* Rv, const PolyPC<T>& pc, T* last_out, const int32_t* flags);
template <typename T>
void launch_cheb_step_t(hipStream_t s, int64_t n, int N, const int32_t* rowptr, const int32_t* col, const T* val,
                        const T* dinv, const T* Rv, const PolyPC<T>& pc, int j, const T* zin, const T* zprev,
                        T* zout, double* part, const int32_t* flags);
void launch_cg_start2(hipStream_t s, int64_t n, int N, const double* partial, double rtol2, const double* mask,
                      double* scal, int32_t* flags, const double* rz_part);
// Direction with an explicit preconditioned residual Zl and its r.z partials
// (spmm_blocks(n, N) of them); null pointers: Jacobi on the fly.
template <typename T>
void launch_cg_direction_z(hipStream_t s, int64_t n, int N, const T* dinv, const T* Rv, T* P, const double* upd_part,
                           const double* scal_in, const int32_t* flags_in, double* scal_out, int32_t* flags_out,
                           double rtol2, const double* rz_part, const T* Zl);
// Two-level correction (one column): eH = KHinv rH (dense); then
// Zout = (Zin or D^-1 R) + P eH and per-block partials of R . Zout
// (spmm_blocks(n, 1) blocks).
void launch_dense_mv(hipStream_t s, int64_t m, const double* Ainv, const double* x, double* y);
void launch_zcoarse(hipStream_t s, int64_t n, const double* dinv, const double* R, const double* Zin,
                    const int32_t* Pk, const double* Pw, const double* eH, double* Zout, double* rz_part);
void launch_gershgorin(hipStream_t s, int64_t n, const int32_t* rowptr, const double* val, const double* dinv,
                       double* partial, double* out);
// cg.hip
int cg_blocks(int64_t n, int N);
int spmm_blocks(int64_t n, int N);
int cg_max_blocks();
void launch_spmm2(hipStream_t s, int64_t n, int N, const int32_t* rowptr, const int32_t* col, const double* val,
                  const double* X, double* Y, double* partial, const int32_t* flags);
void launch_cg_init2(hipStream_t s, int64_t n, int N, const double* B, const double* AX, const double* dinv,
                     double* Rv, double* P, double* partial);
void launch_cg_start(hipStream_t s, int64_t n, int N, const double* partial, double rtol2, const double* mask,
                     double* scal, int32_t* flags);
void launch_spmm2_f32(hipStream_t s, int64_t n, int N, const int32_t* rowptr, const int32_t* col, const float* val,
                      const float* X, float* Y, double* partial, const int32_t* flags);
void launch_cg_init2_f32(hipStream_t s, int64_t n, int N, const float* B, const float* AX, const float* dinv,
                         float* Rv, float* P, double* partial);
void launch_cg_update_f32(hipStream_t s, int64_t n, int N, const float* dinv, float* X, float* Rv, const float* P,
                          const float* Q, const double* pq_part, const double* scal, const int32_t* flags,
                          double* partial, int32_t* brk);
void launch_cg_direction_f32(hipStream_t s, int64_t n, int N, const float* dinv, const float* Rv, float* P,
                             const double* upd_part, const double* scal_in, const int32_t* flags_in, double* scal_out,
                             int32_t* flags_out, double rtol2);
void launch_to_f32(hipStream_t s, int64_t m, const double* a, float* b);
void launch_add_f32(hipStream_t s, int64_t m, const float* d, double* x);
void launch_cg_update_f(hipStream_t s, int64_t n, int N, const double* dinv, double* X, double* Rv, const double* P,
                        const double* Q, const double* pq_part, const double* scal, const int32_t* flags,
                        double* partial, int32_t* brk);
void launch_cg_direction_f(hipStream_t s, int64_t n, int N, const double* dinv, const double* Rv, double* P,
                           const double* upd_part, const double* scal_in, const int32_t* flags_in, double* scal_out,
                           int32_t* flags_out, double rtol2);
// kernels.hip
int elem_blocks(int64_t n, int N);
int qp_blocks(int64_t nt);
int gram_blocks(int64_t n);
int nmom();
// V_ext at npts points (nt x number of quadrature points per tet)
void launch_vext(hipStream_t s, int64_t npts, const double* qpx, const double* RZ, int n_nuclei, int kind,
                 double rc, double omega, double* vext);
void launch_qp_density(hipStream_t s, int64_t nt, const int32_t* tets, const int32_t* v2d, const double* X, int N,
                       const double* occ, double* rho_out);
void launch_qp_fields(hipStream_t s, int64_t nt, const int32_t* tets, const int32_t* v2d, const double* Phi, int N,
                      const double* occ, const double* wnod, const double* vext, const double* geo,
                      const double* qpx, int xck, double xalpha, double* vxc, double* exc, double* veff,
                      double* rho, double* partials);
void launch_reduce_rows(hipStream_t s, const double* partials, int nblk, int nvals, int minlast, double* out);
void launch_boundary_g(hipStream_t s, int64_t nbv, const int32_t* bverts, const double* xyz, const double* mom,
                       double* g);
void launch_field(hipStream_t s, int64_t nt, const int32_t* tets, const double* nod, const int32_t* v2d,
                  const double* dofv, const double* add1, const double* add2, double* out);
// val1 = cK1 K + M_{f1} + cM1 M, val2 = cK2 K + M_{f2} (optional), dinv1 = 1/diag(val1) (optional)
// esl: scratch of 2 ns doubles, 16-byte aligned (ns = slot_ptr[nnz], the element entries in slot order;
// two operators are stored as interleaved pairs).
void launch_assemble2(hipStream_t s, int64_t nt, int64_t n, int64_t nnz, const double* geo, const int32_t* slot_ptr,
                      const int32_t* slot_of, int64_t ns, const int32_t* diag_slot, double* esl, double cK1,
                      const double* f1, double cM1, double* val1, double* dinv1, double cK2, const double* f2,
                      double* val2);
// b = scale * int f phi_a - l_a, l_a = sum over boundary b of K_ab g_b (gnod may be null);
// scratch: 8 nt doubles.
void launch_load(hipStream_t s, int64_t n, int64_t nt, const int32_t* adj_ptr, const int32_t* adj_tet,
                 const int8_t* adj_loc, const int32_t* tets, const double* geo, const double* f_qp, double scale,
                 const double* gnod, const int32_t* v2d, double* scratch, double* b, double* lvec);
// the DoF pass of the load vector (ne nodes per tet, 2 ne element values per tet in scratch)
void launch_load_gather(hipStream_t s, int64_t n, int ne, const int32_t* adj_ptr, const int32_t* adj_tet,
                        const int8_t* adj_loc, const double* scratch, double* b, double* lvec);
// CSR values from the element entries in slot order; dinv = 1 / diagonal
void launch_slot_sum(hipStream_t s, int64_t nnz, const int32_t* slot_ptr, const double* esl, double* val1,
                     double* val2);
void launch_diag_inv(hipStream_t s, int64_t n, const int32_t* diag_slot, const double* val, double* dinv);
void launch_scale_cols_to(hipStream_t s, int64_t n, int N, const double* X, const double* sc, double* Y);
void launch_coldot(hipStream_t s, int64_t n, int N, const double* X, const double* Y, double* partial);
void launch_reduce_cols(hipStream_t s, int N, int nblk, const double* partial, double* out);
// lmax[0] = min(lmax[0], safety x the largest Ritz value of m Lanczos steps on D^-1 A in the D inner
// product); work: 3n doubles; partial: ceil(n / 256) (at most 1024) doubles; scal: 2m + 2 doubles.
void launch_lanczos_lmax(hipStream_t s, int64_t n, const int32_t* rowptr, const int32_t* col, const double* val,
                         const double* dinv, int m, double safety, double* work, double* partial, double* scal,
                         double* lmax);
void launch_normalize_cols(hipStream_t s, int64_t n, int N, const double* sc, double* X);
// P^T Y (nH x N) through the chunk structure: each chunk of RESTRICT_CHUNK
// fine rows of Y is read once (into LDS), its segment sums go to part, then
// the segments of each coarse DoF are summed in chunk order into out.
constexpr int RESTRICT_CHUNK = 128;
// part: the segment partials (nseg x N; null: d.rpart)
void launch_restrict_chunks(hipStream_t s, int64_t n, int64_t nH, int N, const Dev& d, const double* Y, double* out,
                            double* part = nullptr);
void launch_gram(hipStream_t s, int64_t n, int N, const double* U, const double* Y, double* partial);
// chat: per fine tet in coarse-group order e, the parent's coarse hats at its
// quadrature points (16) and its volume: 17 arrays of ng = nt doubles (value
// k of tet e at k ng + e; fixed per mesh).
void launch_coarse_hats(hipStream_t s, int64_t cnt, int64_t ng, const int32_t* grp_ptr, const int32_t* grp_tet,
                        const int32_t* tets, const double* geo, const double* xyz, const double* cgeo, double* chat);
void launch_coarse_ops(hipStream_t s, int64_t cnt, int64_t ng, const int32_t* grp_ptr, const int32_t* grp_tet,
                       const double* chat, const double* cgeo, const double* fA, const double* fW, double* out);
void launch_coarse_orb(hipStream_t s, int64_t cnt, int64_t ng, const int32_t* grp_ptr, const int32_t* grp_dof,
                       const double* chat, const double* U, int N, double* out);
// joint-space variant: (u_j u_l, psi_m) per coarse tet and pair, 4 values each (out: cnt x npair x 4)
void launch_coarse_pairs(hipStream_t s, int64_t cnt, int64_t ng, const int32_t* grp_ptr, const int32_t* grp_dof,
                         const double* chat, const double* U, int N, const int32_t* pair_jl, int npair, double* out);
// Phi = P C + U D (C: nH x N, D: N x N, both row-major)
void launch_reconstruct_joint(hipStream_t s, int64_t n, int N, const int32_t* Pk, const double* Pw, const double* Cc,
                              const double* D, const double* U, double* Phi);
void launch_coarse_tri(hipStream_t s, int64_t cnt, const int32_t* grp_ptr, const int32_t* grp_tet,
                       const int32_t* tets, const double* geo, const double* xyz, const double* cgeo, double* out);
void launch_reconstruct(hipStream_t s, int64_t n, int N, const int32_t* Pk, const double* Pw, const double* phiH,
                        const double* theta2, const double* U, double* Phi);
void launch_hartree_nodal(hipStream_t s, int64_t nv, const int32_t* v2d, const int32_t* Pk, const double* Pw,
                          const double* wH, double theta1, const double* w0, const double* g, double* w);
void launch_rho_nodal(hipStream_t s, int64_t nv, const int32_t* v2d, const double* Phi, int N, const double* occ,
                      double* rho);
// gather = 1: out[a N + i] = in[perm[a] N + i]; gather = 0: out[perm[a] N + i] = in[a N + i]
void launch_permute_rows(hipStream_t s, int64_t n, int N, const int32_t* perm, const double* in, double* out,
                         int gather);
// out[a] = w[d2v[a]] for the n DoFs (interior values of a nodal vector)
void launch_gather_nodal(hipStream_t s, int64_t n, const int32_t* d2v, const double* w, double* out);
// cnt[0] = number of non-finite values in a[0..na) and b[0..nb)
void launch_count_nonfinite(hipStream_t s, int64_t na, const double* a, int64_t nb, const double* b, int32_t* cnt);
// learned initial guess (kernels.hip)
void launch_colmax_abs(hipStream_t s, int64_t n, int N, const double* X, double* partial, double* out);
void launch_features(hipStream_t s, int64_t n, int N, const int32_t* d2v, const double* xyz, const double* w,
                     const double* Phi, const double* AX, const double* B, const double* dinv, const double* occ,
                     const double* RZ, int n_nuclei, int pot, double rc, double omega, int xck, double xalpha,
                     double diag, const double* scale, float* F);
void launch_guess_delta(hipStream_t s, int64_t n, int N, const double* scale, const float* Y, double* D);
void launch_estimate(hipStream_t s, int64_t nt, int N, const int32_t* tets, const int32_t* v2d, const double* Phi,
                     const double* lam, const double* veff, const double* geo, const double* xyz, const int32_t* nbr,
                     const int32_t* tord, double* eta2);
void launch_transfer(hipStream_t s, int64_t m, int64_t first, int64_t nv_old, const int64_t* parents, int ncols,
                     double* values);
// X (= delta on entry) <- Galerkin start in span{Phi, delta} where it lowers J
// and does not raise the residual, Phi elsewhere; gdots: 5N sums; gsel: [used
// (N), |b - A x0|^2 (N), |b - A phi|^2 (N), |b - A X|^2 of the start taken (N)].
void launch_guess_galerkin(hipStream_t s, int64_t n, int N, const double* Phi, const double* AP, const double* AD,
                           const double* B, double* X, double* partial, double* gdots, double* gsel);
void launch_collect(hipStream_t s, int64_t n, int N, int stride, const float* F, const double* U,
                    const double* Phi, const double* scale, int64_t offset, int64_t cap, float* out_x,
                    float* out_t);
void launch_energy(hipStream_t s, int64_t nt, const int32_t* tets, const int32_t* v2d, const double* Phi, int N,
                   const double* occ, const double* wnod, const double* vxc_old, const double* geo, int xck,
                   double xalpha, double* partials);

}  // namespace mlc
