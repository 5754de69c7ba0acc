// Device kernels of the solve path and their host launchers (all asynchronous on
// the given stream).  Layout: cell arrays n^3, index i + n (j + n k), x fastest.
// Batched launches process `nb` arrays at a stride of n^3 elements (leading
// batch index); vectors of the factorizations hold `nb` values per variable
// (variable-major, batch fastest).
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>

#include "fields.hpp"
#include "lu_flow.hpp"

namespace cc {

// Geometry of one level as the stencil kernels see it.
struct StencilLevel {
  int n;
  double inv12h2;        // 1 / (12 h^2)
  int bc[6];             // wall conditions -x,+x,-y,+y,-z,+z (0 Dirichlet, 1 Neumann, 2 Robin)
  double rob[6][2][4];   // Robin walls: the assembled rows (times 12 h^2) of layer 0 and 1 on the 4
                         // cells nearest the wall, nearest first
  const uint8_t* type;   // 0 no unknown, 1 phi_1, 2 phi_2
  int march;             // regular-row kernels (SMO-1, residual, apply): 1 march in z, 2 march in z with the
                         // XCD-aware tile order, 0 one cell per thread
  int kz;                // planes per workgroup of the marching kernels
  const uint8_t* zone;   // 1: a phi_2 cell or a phi_1 cell whose row reads within 3 cells of one (the far
                         // sweep leaves these to the near sweep); null on levels without phi_2 cells
};

// The build's choice of the regular-row kernel schedule for an n^3 level.
void default_stencil_schedule(int n, int& march, int& kz);

// FV-PLG rows of one level, ELL layout (entry j of row r at j * N2 + r).
struct PlgRows {
  int N2;
  const int* cell;        // N2 target cells
  const int* cols;        // 35 * N2 stencil cells
  const double* vals;     // 35 * N2 coefficients
  const float* vals32;    // the same rounded to FP32 (mixed precision; may be null)
  const uint64_t* phi2;   // N2 masks: bit j set if entry j is a phi_2 cell
  const int* nd;          // N2: position of row r in the level's factorization order
};

// Supernodal factors and work vectors of one factorization, in FP64 and (for
// mixed precision) FP32 copies.
struct LuDev {
  int n;                 // variables
  const int* var_cell;   // n: grid cell of each variable (ND order)
  const int* row_cell;   // n: grid cell of the equation stored at each position
  const double* M;
  const double* V;
  const double* W;
  const float* M32;
  const float* V32;
  const float* W32;
  const int* U;           // later variables of each node (backward)
  const int* Uf;          // their equation positions in pivot order (forward)
  double* y;              // work vectors, n * nb values (FP64)
  double* z;
  double* x;
  float* y32;             // FP32 work vectors
  float* z32;
  float* x32;
};

// Task lists of one height of a factorization's tree (the heights run as
// successive launches).  A single-RHS task is one wavefront taking 64/g rows
// of one node with g lanes per row (lg = log2 g); a multi-RHS task is one
// wavefront taking up to kMrRows rows of one node, one lane per right-hand
// side.  Forward rows are those of [L11^-1 ; L21 L11^-1] (p + q rows), whose
// L21 part is accumulated atomically into the later equations; backward rows
// are those of [U11^-1 | U11^-1 U12] (p rows).
struct LuTask {
  long long offM;         // node's M block
  long long offVW;        // node's V block (forward) or W block (backward)
  long long offU;         // node's later-variable list
  int base, p, q;         // node's first variable, size, later variables
  int row0, lg, pad;      // first row of this task, log2 lanes per row
};
constexpr int kMrRows = 4;
// Single-RHS tasks load a row's entries kc per lane at a time (kc 4 or 8, all
// loads of a round in flight together), so a task whose rows hold at most kc
// entries per lane waits on one memory round trip.
struct LuTasks {
  int nF, nB;             // single-RHS forward / backward tasks
  int kc = 8;             // entries per lane per load round
  int wcap = 1 << 30;     // single RHS: at most this many wavefronts per launch
  const LuTask* ftask;
  const LuTask* btask;
  int nFm, nBm;           // multi-RHS forward / backward tasks
  const LuTask* ftask_m;
  const LuTask* btask_m;
};

// The lower heights of the tree as subtrees, one workgroup each: for subtree s,
// levels lptr[s] .. lptr[s+1] of lev, each a task range [x, y) of one height
// (forward: heights ascending; backward: descending).
struct LuSubList {
  const LuTask* ftask;
  const int2* flev;
  const int* fptr;
  const LuTask* btask;
  const int2* blev;
  const int* bptr;
};
struct LuSub {
  int nsub = 0;           // subtrees (0: no subtree launch)
  int hcut = 0;           // heights below hcut belong to the subtrees
  int kc = 8;             // entries per lane per load round (single RHS)
  LuSubList single{}, multi{};
};

// One launch per sweep (single right-hand side; protocol in lu_flow.hpp): the
// forward tasks of every height in ascending height order, each waiting on its
// node's children; the backward tasks in descending order, each waiting on its
// node's parent.
struct LuFlow {
  FlowGraph fwd{}, bwd{};
  const LuTask* ftask = nullptr;  // fwd.ntask tasks in ticket order
  const LuTask* btask = nullptr;  // bwd.ntask tasks in ticket order
  int* counters = nullptr;        // fwd.done, bwd.done and the two tickets: zeroed before each solve
  int ncounters = 0;
  int* err = nullptr;             // nonzero once a wait gave up (checked and cleared by the host)
  int kc = 8;                     // entries per lane per load round
  long long limit = 0;            // wait bound in wall-clock ticks
  int max_waves = 0;              // wavefronts of a sweep launch at most (0: enough to fill the chip)
};

// ---- stencil work (T = double or float), nb arrays at stride n^3
template <class T>
void launch_smo1(const StencilLevel& L, double omega, const T* s, const T* e_in, T* e_out, int nb, hipStream_t st);
// first sweep of a level from e = 0: e_out = omega D^-1 s on phi_1 cells, 0 elsewhere
template <class T>
void launch_smo1_first(const StencilLevel& L, double omega, const T* s, T* e_out, int nb, hipStream_t st);
// SMO-1 split in two for overlap with the LU-correction: the far sweep writes
// every cell whose zone is 0 (phi_1 rows that read no phi_2 cell, and cells
// without an unknown, passed through), the near sweep the listed phi_1 cells of
// zone 1 (phi_2 cells are left alone: the next SMO-2 overwrites them).  Both
// compute exactly what launch_smo1 computes for their cells.
template <class T>
void launch_smo1_far(const StencilLevel& L, double omega, const T* s, const T* e_in, T* e_out, int nb,
                     hipStream_t st);
template <class T>
void launch_smo1_near(const StencilLevel& L, double omega, const T* s, const T* e_in, T* e_out, const int* cells,
                      int count, int nb, hipStream_t st);
template <class T>
void launch_restrict(const StencilLevel& F, const StencilLevel& C, const T* s, const T* e, T* sc, int nb,
                     hipStream_t st);
template <class T>
void launch_prolong_add(const StencilLevel& F, int nc, const T* ec, T* ef, int nb, hipStream_t st);
// full multigrid transfers (FP64, nb arrays): right-hand side restriction
// (children with an unknown averaged) and renormalised trilinear interpolation
void launch_fmg_restrict(const StencilLevel& F, const StencilLevel& C, const double* s, double* sc, int nb,
                         hipStream_t st);
void launch_fmg_prolong(const StencilLevel& F, const StencilLevel& C, const double* xc, double* xf, int nb,
                        hipStream_t st);
template <class T>
void launch_plg_b2(const PlgRows& P, const T* s, const T* e, T* y, long long stride, int nb, hipStream_t st);
template <class T>
void launch_zero(T* p, long long count, hipStream_t st);

// ---- FP64 outer residual and apply
void launch_stencil_residual(const StencilLevel& L, const double* r, const double* x, double* s, int nb,
                             hipStream_t st);
void launch_stencil_apply(const StencilLevel& L, const double* x, double* y, hipStream_t st);
void launch_plg_residual(const PlgRows& P, const double* r, const double* x, double* s, int apply_only, int nb,
                         long long stride, hipStream_t st);

// ---- factorizations: T is the factor and work-vector type, TO the output array
// type.  y (work vector) gathers src at the stored equation cells.
template <class TS, class TY>
void launch_gather(int n, const int* row_cell, const TS* src, long long src_stride, TY* y, int nb, hipStream_t st);
template <class T>
void launch_lu_forward(const LuDev& F, const LuTasks& S, int nb, hipStream_t st);
template <class T, class TO>
void launch_lu_backward(const LuDev& F, const LuTasks& S, TO* out, long long out_stride, int nb, hipStream_t st);
template <class T>
void launch_lu_forward_sub(const LuDev& F, const LuSub& S, int nb, hipStream_t st);
template <class T, class TO>
void launch_lu_backward_sub(const LuDev& F, const LuSub& S, TO* out, long long out_stride, int nb, hipStream_t st);
// one LU solve as a counter reset and two launches (single right-hand side)
template <class T, class TO>
void launch_lu_flow(const LuDev& F, const LuFlow& W, TO* out, hipStream_t st);

// ---- norms, updates, fills (nb arrays; norms are nb u64 bit patterns of
// non-negative doubles, combined by atomicMax)
void launch_zero_u64(unsigned long long* p, int count, hipStream_t st);
// out[b] = bit pattern of max |v_b| (non-negative doubles order like unsigned
// integers); partial: kReductionScratch doubles of scratch
constexpr int kReductionScratch = 2048 * 64;
void launch_maxabs(const double* v, long long count, int nb, unsigned long long* out, double* partial,
                   hipStream_t st);
// phi += scale_b * e on unknown cells; scale_b = norm[b] (or 1 if norm is null)
template <class T>
void launch_add_unknowns(const StencilLevel& L, const T* e, const unsigned long long* norm, double* phi, int nb,
                         hipStream_t st);
// d = s / norm[b] (0 where norm[b] == 0), converted to T
template <class T>
void launch_scale_residual(long long n3, const double* s, const unsigned long long* norm, T* d, int nb,
                           hipStream_t st);
void launch_mask_unknowns(const StencilLevel& L, double* a, int nb, hipStream_t st);
// a[pair.x] = a[pair.y] for every pair (merged cell <- its host), nb arrays
template <class T>
void launch_copy_pairs(int count, const int2* pairs, T* a, long long stride, int nb, hipStream_t st);
void launch_cell_average(int n, double h, const double* origin, const FieldDesc& f, int mode, int q,
                         double* out, hipStream_t st);
// One line piece of a cut cell's volume rule (the layout of cc::LinePiece): q
// Gauss points on [a, b] along axis k at the base point xo (the other two
// coordinates in ascending axis order), weights w (b - a)/2 w_j.
struct PieceRec {
  double xo[2];
  double a, b, w;
  int k, pad;
};
// out[c * nf + f] = the q-point rules of the pieces off[c] .. off[c+1]-1 of cell
// c applied to field f (mode 0 value, 1 Laplacian) for ncell cells and nf
// device-resident field descriptors; one workgroup per (cell, group of up to 8
// fields).
void launch_piece_integrals(int ncell, const int* off, const PieceRec* pieces, int q, const FieldDesc* fds, int nf,
                            int mode, double* out, hipStream_t st);
void launch_set_values(int count, const int* cells, const double* vals, double* a, hipStream_t st);
// a[b * stride + cells[v]] = vals[v * nb + b] (add = 0) or += it (add = 1), nb arrays
void launch_scatter_values(int count, const int* cells, const double* vals, double* a, long long stride, int nb,
                           int add, hipStream_t st);
void launch_copy(long long count, const double* src, double* dst, hipStream_t st);
// Krylov helpers over n3-element FP64 vectors stored `stride` apart (partial:
// reduction scratch as for launch_maxabs):
// out = / += / -= sum_i coef_i V_i (mode 0 / 1 / 2; coef on the device), with
// optional max |out| into *amax (bit pattern) and sum of out^2 into *sumsq;
// out[i] = (w, V_i) for i < nv and out[nv] = (w, w), w read once per 8 vectors
void launch_combo(long long n3, const double* V, long long stride, int nv, const double* coef, double* out, int mode,
                  unsigned long long* amax, double* sumsq, double* partial, hipStream_t st);
void launch_dots_norm(long long n3, const double* w, const double* V, long long stride, int nv, double* out,
                      double* partial, hipStream_t st);
// learned guess: coarse features (block mean of r scaled, volume fraction) and
// trilinear prolongation of the network output to the level-0 unknowns
void launch_net_features(int n0, int m, const double* r, double inv_norm, const float* volfrac, float* x,
                         hipStream_t st);
// training pairs (features, targets, mask) of nb solved problems on an m^3 level
void launch_net_pairs(int n0, int m, int nb, const double* r, const double* phi, const uint8_t* type0,
                      const unsigned long long* norm, const float* volfrac, double phi_scale, float* x, float* t,
                      uint8_t* mask, hipStream_t st);
void launch_prolong_trilinear(const StencilLevel& L0, int m, const float* y, double scale, double* phi,
                              hipStream_t st);
// x = scale y on the unknown cells of level Lm (n_m^3 cells), 0 elsewhere
void launch_net_to_level(const StencilLevel& Lm, const float* y, double scale, double* x, hipStream_t st);

// FV-PLG weighted least-squares fits on the device (setup): nsys systems, system
// s the rows off[s] .. off[s+1] of A (35 doubles each, weighted); y receives the
// minimum-norm solutions of A_s^T y = ell_s, ok[s] = 0 for a rank-deficient A_s.
// Host arrays; allocates device buffers, synchronises st.
void plg_lsq_device(int nsys, const int* off, const double* A, const double* ell, double* y, int* ok,
                    hipStream_t st);

// Scratch of the allocation-free entry points: one fixed device array per GPU
// (kNoAllocScratchDoubles doubles, held until the process ends).  The first call
// on a device, with that device current, resolves the array's device address
// on it (hipGetSymbolAddress) and keeps it; later calls return the kept
// address.  Throws cc::Error(CC_EDEVICE) if the address cannot be resolved.
constexpr long long kNoAllocScratchDoubles = 6LL << 20;   // 48 MiB
void noalloc_scratch(int device, double** ptr, long long* capacity);

}  // namespace cc
