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
  const double* M;
  const double* V;
  const double* W;
  const int* U;
  const int* piv;        // per node: absolute variable of pivoted row j
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

// Task lists of one height: F-row tasks (node, row) and variable tasks.
struct LuTasks {
  int nF;                 // F-row tasks
  const int2* ftask;      // (node, row)
  int nVar;               // forward variable tasks
  const int* vvar;        // variable index
  const int* vptr;        // nVar + 1
  const int2* ventry;     // (node, row of V)
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
void launch_lu_forward(const LuDev& F, const LuTasks& T, hipStream_t st);
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
