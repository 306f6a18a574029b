// Launch descriptors and host launchers of every kernel of the library.
#pragma once

#include "wc_fields.h"

namespace wc {

constexpr int NKV_MAX = 32;   // largest FGCR restart length
constexpr int HIST_MAX = 64;  // restarts whose true residual a solve reports

// ----------------------------------------------------------------- D_w
struct DiracLaunch {
  const LatDesc* lats;
  const WorkItem* items;
  int nitems;
  const void* in;
  const float* in_sc;
  void* out;
  float* out_sc;
  const void* y;       // if set: out = y - D in (same precision as out)
  const float* y_sc;
  double* partials;    // if set: |out|^2 per (system, chunk), stride pw
  int pw;
  const int* skip;     // if set: systems with skip != 0 are not written
  int dagger;          // apply gamma5 D gamma5
  int block;           // Dirichlet-block operator instead of the full one
  int stage;           // the items' lattices have 256-site tiles: stage each tile's input in LDS
  int in_prec;         // storage precision of `in` (may differ from the launch's for FP64 and FP32)
  // FGCR cycle: dead[0] != 0 once every system has ended the cycle (the launch then does
  // nothing).  The block solvers do not take it: the check alone moved scalar-register spill
  // code into the even/odd solver's MR loop (+13 instructions per step, half-sweep 1538 ->
  // 1566 us), more than their launches after the end of a cycle cost
  const int* dead = nullptr;
};
void launch_dirac(int prec, int nr, const DiracLaunch& a, int grid, hipStream_t st);
// a launch of an FGCR cycle after every system has ended it
WC_D bool cycle_dead(const int* dead) { return dead && gld_i32(dead, 0) != 0; }
size_t dirac_stage_lds_bytes(int prec, int nr);  // dynamic LDS of a staged D_w launch
constexpr size_t LDS_MAX_BYTES = 160 * 1024;       // LDS a gfx950 work-group may allocate

// ----------------------------------------------------------------- Schwarz block MR
struct SapLaunch {
  const LatDesc* lats;
  const WorkItem* items;  // chunk = index into the colour's tile list
  int nitems;
  int colour;
  int nmr;
  void* rho; float* rho_sc;
  void* z; float* z_sc;
  void* psi; float* psi_sc;
  const int* skip;
  int first;        // psi = z (else psi += z)
  int border;       // subtract the hops out of the other colour's z before solving
  int write_rho;
  int write_z;
  int cache;        // keep links and clover in registers across the MR steps (FP32 math only)
  int uniform_bvol; // block volume shared by every lattice of the launch (0 if they differ)
  // even/odd solver, residual on odd sites (zero after every solve of the block):
  // 0 read and stored, 1 read but not stored, 2 neither read (taken as zero) nor stored
  int odd_rho;
  // even/odd solver: the border update's cross-block hops as LDS entries (border_entries =
  // the largest count of any lattice of the launch; 0 = per-site path), after the exchange
  // rows of length eo_rows
  int border_entries;
  int eo_rows;
};
void launch_sap_mr(int prec, int nr, const SapLaunch& a, int grid, int block_threads, hipStream_t st);
size_t sap_lds_bytes(int prec, int nr, int bvol);
// 16-bit storage, 4^4 blocks: block operator staged in LDS and shared by nr (1 or 2) rhs
void launch_sap_mr_lds(int prec, int nr, const SapLaunch& a, int grid, hipStream_t st);

// even/odd-preconditioned block solver: two lanes per (even site, odd site) pair of a block
void launch_sap_eo(int prec, int nr, const SapLaunch& a, int grid, int max_bvol, hipStream_t st);
// dynamic LDS of the even/odd solver: reduction scratch, the exchange rows and, when
// border_entries > 0, the border update's entries
size_t sap_eo_lds_bytes(int prec, int nr, int max_bvol, int border_entries);
// cross-block hops of one block (the border update's entries): two faces per direction
WC_HD int border_entry_count(const int* B) {
  const int vol = B[0] * B[1] * B[2] * B[3];
  return 2 * (vol / B[0] + vol / B[1] + vol / B[2] + vol / B[3]);
}

// ----------------------------------------------------------------- layout conversion / setup
// canonical complex128 [rhs][V][4][3] (lexicographic) <-> internal field of one lattice
void launch_pack_spinor(int prec, const Geom& g, int nrhs, const void* canon, void* dst, float* dst_sc,
                        hipStream_t st);
void launch_unpack_spinor(int prec, const Geom& g, int nrhs, const void* src, const float* src_sc, void* canon,
                          int colour_only, hipStream_t st);
// canonical complex128 links [4][V][3][3] -> internal links
void launch_pack_links(int prec, const Geom& g, const void* canon, void* dst, float* dst_sc, hipStream_t st);
// clover blocks from internal FP64 links, FP64 storage
void launch_clover_build(const Geom& g, const void* links64, double m0, double csw, void* clov64, hipStream_t st);
// even/odd block-solver clover: A on even sites, A^-1 on odd sites (FP64 -> FP64)
void launch_clover_eo(const Geom& g, const void* clov64, void* out64, hipStream_t st);
// FP64 clover -> storage precision
void launch_clover_convert(int prec, const Geom& g, const void* clov64, void* dst, float* dst_sc, hipStream_t st);

// ----------------------------------------------------------------- FGCR vector kernels
struct SysState {
  double bnorm2;
  double rnorm2;       // |r|^2, recursive inside a cycle, true after a restart
  double thr2;         // cycle stops once rnorm2 <= thr2
  double cyc2;         // ... or once rnorm2 <= cyc2 (drop^2 x the true |r|^2 the cycle started from)
  double tol2;         // solve stops once the true |r|^2 <= tol2
  int cycle_done;
  int converged;
  int k_done;
  int iters;
  int restarts;
  int breakdown;
  double sap_scale;    // |r| at the current SAP input
  int reorth;          // the current direction takes a second Gram-Schmidt pass
  int reorths;         // second passes taken in this solve
  double n2_first;     // |chi_k|^2 before the first pass
  double prev_true2;   // true |r|^2 of the previous restart (stagnation test)
  int stall;           // consecutive restarts whose true residual did not drop
  int stagnated;       // the solve stopped because the true residual stagnated
  double2 a[NKV_MAX * NKV_MAX];  // a[l * NKV_MAX + k] = <chi_l, chi_k> (both passes)
  double2 e[NKV_MAX];            // <chi_l, r> at the current iteration
  double2 a2[NKV_MAX];           // second-pass coefficients of the current iteration
  double bk[NKV_MAX];
  double2 ck[NKV_MAX];
  double2 alpha[NKV_MAX];
};

// FGMRES-DR state per system: the cycle's (m+1) x m matrix Hbar, its Givens rotations and
// rotated residual coefficients g (|g[j+1]| = least-squares residual after column j), and
// the deflation basis P used to recombine V and Z at a restart.
constexpr int ARN_LD = NKV_MAX + 1;
constexpr int ARN_ROT_MAX = NKV_MAX * (NKV_MAX + 1) / 2 + NKV_MAX + 1;
struct ArnState {
  int nrot;      // rotations in use
  int lucky;     // the last new basis vector was (numerically) zero: invariant subspace
  int pin, pout; // P is pin x pout
  double2 H[ARN_LD * NKV_MAX];  // column-major, leading dimension ARN_LD
  double2 g[ARN_LD];
  double rc[ARN_ROT_MAX];
  double2 rs[ARN_ROT_MAX];
  int rp[ARN_ROT_MAX];
  double2 P[ARN_LD * ARN_LD];   // column-major, leading dimension ARN_LD
  double2 h1[ARN_LD], h2[ARN_LD];  // the two Gram-Schmidt passes' coefficients of column j
  double w2;                       // |w|^2 before the first pass
};

struct VecLaunch {
  const LatDesc* lats;
  const WorkItem* items;   // nr = 1
  int nitems;
  SysState* sys;
  int* skip;               // per system: 1 while it sits out the current cycle
  double* partials;        // [total_chunks][pw]
  int pw;
  int k;                   // iteration index inside the cycle
  int maxit;               // cap on FGCR iterations per system
  double tol;              // relative residual target
  int stag;                // restarts in a row without a drop of the true residual that stop
                           // a system (0: never)
  double* hist;            // [nsys][hist_max] relative true residual after each restart (or null)
  int hist_max;
  // F64 batched fields
  double2* r;
  double2* x;
  double2* const* chi;     // device array of NKV_MAX pointers
  double2* const* phi;
  // SAP-precision field for conversions
  void* sp; float* sp_sc;
  ArnState* arn;           // FGMRES-DR state per system (null for FGCR)
  // FGCR: the search directions phi_l as the preconditioner wrote them (storage dir_prec,
  // device arrays of NKV_MAX data / scale pointers), and whether the residual update also
  // writes the next preconditioner input r / |r_k| into sp (all but a cycle's last step)
  void* const* dir;
  float* const* dir_sc;
  int dir_prec;
  int fuse_sap;
  // FGCR Krylov basis chi_l (device array of NKV_MAX pointers, storage F64 or F32) and the
  // current direction D phi_k before its Gram-Schmidt, in the basis storage (with an FP64
  // basis, chi_k itself: the update then overwrites it in place)
  void* const* q;
  void* w;
  void* rq;                // the recursion's residual in the basis storage (with an FP64 basis, r)
  // FGCR cycle: [0] != 0 once every system has ended the cycle (the residual-norm reduction
  // sets it, the cycle's first conversion clears it; D and Gram-Schmidt then do nothing), [1] and
  // [2] that reduction's arrival and ended-system counts (zero between launches); or null
  int* dead;
  double drop2;            // a cycle ends once |r|^2 <= drop2 x its starting true |r|^2 (0: never)
};
// eta(P) = r / |r|, the preconditioner's input at the start of a restart cycle (later
// steps get theirs from the residual update); the FGCR direction phi_k is the
// preconditioner's output as stored (GCR is invariant to the scale of a direction)
// (with an F32 basis also the recursion's F32 residual rq = r, rounded)
void launch_to_sap(int prec, int basis_prec, const VecLaunch& a, int grid, hipStream_t st);
// Gram-Schmidt kernels for a basis stored in basis_prec (P_F64 or P_F32)
void launch_gs_dots(int basis_prec, const VecLaunch& a, int grid, hipStream_t st);  // <chi_l, w>, <chi_l, r>, |w|^2, <w, r>
// chi_k = (w - sum a_lk chi_l)/b_k in the basis storage; r -= c_k chi_k (chi_k as stored);
// |r|^2.  A system whose first pass cancelled (reorth) instead keeps w - sum a_lk chi_l in w
// and its second-pass dots, and launch_gs_update2 finishes it after the RED_GS2 reduction.
void launch_gs_update(int sap_prec, int basis_prec, const VecLaunch& a, int grid, hipStream_t st);
void launch_gs_update2(int sap_prec, int basis_prec, const VecLaunch& a, int grid, hipStream_t st);
void launch_x_update(const VecLaunch& a, int grid, hipStream_t st);     // x += sum alpha_l phi_l (FP64 phi)
void launch_x_update_dir(const VecLaunch& a, int grid, hipStream_t st); // x += sum alpha_l dir_l
void launch_norm2(const VecLaunch& a, const double2* v, int grid, hipStream_t st);  // |v|^2 partials
void launch_copy_f64(const VecLaunch& a, double2* dst, const double2* src, int grid, hipStream_t st);
void launch_zero_if_b0(const VecLaunch& a, double2* x, int grid, hipStream_t st);  // x = 0 where |b| = 0

// per-system reductions and scalar steps (one work-group per system)
enum ReduceOp { RED_GS = 1, RED_RNORM = 2, RED_TRUE = 3, RED_BNORM = 4, RED_INITR = 5, RED_GS2 = 6 };
void launch_reduce(int op, const VecLaunch& a, int nsys, const int* sys_part, const int* sys_nchunks,
                   hipStream_t st);
void launch_backsub(const VecLaunch& a, int nsys, hipStream_t st);

// ----------------------------------------------------------------- FGMRES-DR (Arnoldi in FP64)
// a.chi = basis V (m+1 entries), a.phi = preconditioned directions Z, a.k = column j
void launch_arn_init(const VecLaunch& a, int grid, hipStream_t st);               // V_0 = r / |r|
void launch_arn_to_sap(int prec, const VecLaunch& a, int grid, hipStream_t st);   // eta(P) = V_j
void launch_arn_from_sap(int prec, const VecLaunch& a, int grid, hipStream_t st); // Z_j = psi
// Gram-Schmidt twice: dots (h1 = <V_i, w>), reduce pass 1, w -= sum h1_i V_i with the
// second pass's dots fused (h2 = <V_i, w>, |w|^2), reduce pass 2 (column j of Hbar = h1 + h2,
// h_{j+1,j}, Givens, stop test), then V_{j+1} = (w - sum h2_i V_i) / h_{j+1,j}
void launch_arn_dots(const VecLaunch& a, int grid, hipStream_t st);
void launch_arn_reduce(int pass, const VecLaunch& a, int nsys, const int* sys_part, const int* sys_nchunks, int m,
                       hipStream_t st);
void launch_arn_update1(const VecLaunch& a, int grid, hipStream_t st);
void launch_arn_update(const VecLaunch& a, int grid, hipStream_t st);
// V_l <- sum_i P_il V_i (l < pout, i < pin), Z_l <- sum_i P_il Z_i (l < pout-1, i < pin-1), in place
void launch_arn_recombine(const VecLaunch& a, int grid, hipStream_t st);

// ----------------------------------------------------------------- force
// K_mu(x) += coef * d Re<Y, D X>/dU (torch convention: G = K^dag) per link, canonical [4][V][3][3]
void launch_link_grad(const Geom& g, const void* links64, const void* Y, const void* X, int nrhs, double csw,
                      double coef, void* Kout, hipStream_t st);
void launch_lie_force(const Geom& g, const void* links64, const void* K, void* F, hipStream_t st);

}  // namespace wc
