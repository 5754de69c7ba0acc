// Device kernels of the solve path and their host launchers (all asynchronous on
// the given stream).  Layout: cell arrays n^3, index i + n (j + n k), x fastest.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>

#include "fields.hpp"

namespace cc {

// Geometry of one level as the stencil kernels see it.
struct StencilLevel {
  int n;
  double inv12h2;        // 1 / (12 h^2)
  int bc[6];             // wall conditions -x,+x,-y,+y,-z,+z
  const uint8_t* type;   // 0 no unknown, 1 phi_1, 2 phi_2
};

// FV-PLG rows of one level, ELL layout (entry j of row r at j * N2 + r).
struct PlgRows {
  int N2;
  const int* cell;        // N2 target cells
  const int* cols;        // 35 * N2 stencil cells
  const double* vals;     // 35 * N2 coefficients
  const uint64_t* phi2;   // N2 masks: bit j set if entry j is a phi_2 cell
  const int* nd;          // N2: position of row r in the level's factorization order
};

// Supernodal factors and the per-height task lists of one factorization.
struct LuDev {
  int n;                 // variables
  const int* var_cell;   // n: grid cell of each variable (ND order)
  const int* row_cell;   // n: grid cell of the equation stored at each position
  const double* M;
  const double* V;
  const double* W;
  const int* U;           // later variables of each node (backward)
  const int* Uf;          // their equation positions in pivot order (forward)
  const int* nbase;
  const int* np;
  const int* nq;
  const long long* offM;
  const long long* offV;
  const long long* offW;
  const long long* offU;
  const long long* offPiv;
  double* y;             // work vectors (n)
  double* z;
  double* x;
};

// Task lists of one height.  A task is one wavefront: (node, first row,
// log2 g, unused) taking 64/g rows with g lanes per row.  Forward rows are those
// of [L11^-1 ; L21 L11^-1] (p + q rows); their L21 part is accumulated
// atomically into the later equations.  Backward rows are those of
// [U11^-1 | U11^-1 U12] (p rows).
struct LuTask {
  long long offM;         // node's M block
  long long offVW;        // node's V block (forward) or W block (backward)
  long long offU;         // node's later-variable list
  int base, p, q;         // node's first variable, size, later variables
  int row0, lg, pad;      // first row of this task, log2 lanes per row
};
struct LuTasks {
  int nF;                 // forward tasks
  const LuTask* ftask;
  int nB;                 // backward tasks
  const LuTask* btask;
};

void launch_smo1(const StencilLevel& L, double omega, const double* s, const double* e_in, double* e_out,
                 hipStream_t st);
void launch_stencil_residual(const StencilLevel& L, const double* r, const double* x, double* s, hipStream_t st);
void launch_stencil_apply(const StencilLevel& L, const double* x, double* y, hipStream_t st);
void launch_plg_residual(const PlgRows& P, const double* r, const double* x, double* s, int apply_only,
                         hipStream_t st);
void launch_restrict(const StencilLevel& F, const StencilLevel& C, const double* s, const double* e,
                     double* sc, hipStream_t st);
void launch_prolong_add(const StencilLevel& F, int nc, const double* ec, double* ef, hipStream_t st);
void launch_plg_b2(const PlgRows& P, const double* s, const double* e, double* y, hipStream_t st);
void launch_gather(int n, const int* var_cell, const double* src, double* y, hipStream_t st);
void launch_lu_forward(const LuDev& F, const LuTasks& T, hipStream_t st);  // GEMV tasks + reduction
void launch_lu_backward(const LuDev& F, const LuTasks& T, double* out, hipStream_t st);
void launch_zero(double* p, long long count, hipStream_t st);
void launch_zero_u64(unsigned long long* p, hipStream_t st);
void launch_maxabs(const double* v, long long count, unsigned long long* out, hipStream_t st);
void launch_add_unknowns(const StencilLevel& L, const double* e, double* phi, hipStream_t st);
void launch_copy_pairs(int count, const int2* pairs, double* a, hipStream_t st);
void launch_cell_average(int n, double h, const double* origin, const FieldDesc& f, int mode, int q,
                         double* out, hipStream_t st);
void launch_set_values(int count, const int* cells, const double* vals, double* a, hipStream_t st);
void launch_mask_unknowns(const StencilLevel& L, double* a, hipStream_t st);

}  // namespace cc
