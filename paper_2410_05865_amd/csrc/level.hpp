// Host construction of one grid level (Secs. 2.2-2.4, 4.1-4.2): cell
// classification and moments, merging, the phi_1/phi_2 split, FV-PLG stencils
// and their weighted least-squares rows, and the sparse blocks the solver needs.
#pragma once
#include <cstdint>
#include <map>
#include <vector>

#include "common.hpp"
#include "fields.hpp"
#include "quadrature.hpp"

namespace cc {

struct Obstacle {
  double c[3], axes[3], rot[9];
  int bc;
  double alpha = 1.0, beta = 0.0;  // CC_ROBIN: alpha phi + beta dphi/dn = g
  int kind = 0;                    // CC_ELLIPSOID or CC_TORUS
  double radii[2] = {0.0, 0.0};    // CC_TORUS: major and minor radius
  double R;   // bounding-sphere radius
  LevelSet ls;  // positive in Omega
};

struct DomainSpec {
  int n;
  double origin[3];
  double h;
  int wall_bc[6];
  double wall_robin[6][2] = {};  // (alpha, beta) of CC_ROBIN walls
  std::vector<Obstacle> obst;
  bool inside = false;  // Omega = interior of obst[0] (its quadric negated: Omega = {ls > 0} either way)
};

enum : int8_t { kExterior = 0, kInterior = 1, kCut = 2 };
enum : uint8_t { kNone = 0, kPhi1 = 1, kPhi2 = 2 };

struct CutData {
  int obst;
  double vol;          // absolute
  double m[N4];        // <xi^a> over the cut cell, own frame
  double area;         // absolute patch area
  double sm[N4];       // <<xi^a>> over the patch
  double sn[3][N3];    // <<n_d xi^a>> over the patch, |a| <= 3
};

// A boundary site of an FV-PLG row: irregular patch of cut cell `cell`
// (kind 'S') or the wall face (axis, side) of a stencil cell (kind 'W').
struct Site {
  int row;        // phi_2 row index
  char kind;
  int cell;
  int bc;
  int axis, side;
  double coef;    // coefficient of the site datum in the row
};

constexpr int kPLG = 35;

// Batched solver of the FV-PLG weighted least-squares problems: for system s
// (rows off[s] .. off[s+1] of A, each 35 doubles, already scaled by the square
// roots of the weights) the minimum-norm y with A^T y = ell[35 s ..], written
// to y[off[s] ..]; ok[s] = 0 where A is rank-deficient (a diagonal entry of R
// below 1e-13 times max |A|).  Used by LevelHost::build when given.
struct PlgLsqSolver {
  virtual void solve(int nsys, const int* off, const double* A, const double* ell, double* y, int* ok) = 0;
  virtual ~PlgLsqSolver() = default;
};

// The assembled regular row next to one wall (coefficients times 12 h^2):
// layer 0 (the cell on the wall) and layer 1, each on the 4 cells nearest the
// wall (nearest first, A_1..A_4), and the coefficient of the wall datum
// (Dirichlet <g>, Neumann <dphi/dn>, Robin <alpha g + beta dg/dn>; n outward).
// Built from the two ghost-cell formulas beyond the wall (Sec. 2.3).
struct WallRows {
  double lay[2][4];
  double dat[2];
};
WallRows wall_rows(int bc, double alpha, double beta, double h);

struct LevelHost {
  int n = 0;
  double h = 0, origin[3] = {0, 0, 0};
  int wall_bc[6] = {};
  WallRows wall[6] = {};
  const DomainSpec* dom = nullptr;

  std::vector<int8_t> cls;       // n^3
  std::vector<double> vol;       // n^3 absolute volume
  std::vector<int> owner;        // n^3 obstacle claiming the cell, -1 if none
  std::map<int, CutData> cut;    // cut cells
  std::vector<int> host;         // n^3: -1 exterior, else the cell carrying the unknown
  std::map<int, std::vector<int>> groups;  // hosts of merged groups -> sorted members
  std::vector<uint8_t> plain;    // n^3 plain interior unknown
  std::vector<uint8_t> type;     // n^3 kNone / kPhi1 / kPhi2
  std::vector<int> unknowns;     // sorted cells carrying an unknown
  std::vector<int> phi2;         // sorted phi_2 cells (row order)
  std::vector<int> plg_cols;     // N2 x 35 stencil cells (lattice order)
  std::vector<double> plg_vals;  // N2 x 35 coefficients (include 1/h^2)
  std::vector<Site> sites;       // boundary sites of all rows
  long long n_merged = 0;

  int idx(int i, int j, int k) const { return i + n * (j + n * k); }
  void ijk(int p, int& i, int& j, int& k) const {
    i = p % n;
    j = (p / n) % n;
    k = p / (n * n);
  }
  const std::vector<int>& members(int p, std::vector<int>& tmp) const;

  // lsq: where the FV-PLG fits run (null: on the host)
  void build(const DomainSpec& d, int n_level, double theta, PlgLsqSolver* lsq = nullptr);

  // Regular-row wall data term of a phi_1 cell: coefficients multiplying the wall
  // datum of each (axis, side) it touches; used by the right-hand side.
  double face_area(int p, int d, int side) const;

 private:
  void claim();
  void classify();
  void merge(double theta);
  void split();
  void rows(PlgLsqSolver* lsq);
  bool regular_ok(int p) const;
  void plg_select(int p, int cells[kPLG]) const;
  // the weighted system of the row of phi_2 cell p: M (m x 35, row-major, rows
  // scaled by sw), sw (m), ell (35), the boundary sites (coef unset)
  void plg_system(int p, int row, const int cells[kPLG], std::vector<double>& M, std::vector<double>& sw,
                  double ell[N4], std::vector<Site>& sites) const;
  void group_moments(int target, int cell, double out[N4]) const;
};

// Binomial shift of own-frame moments to a frame displaced by delta (grid units):
// out_a = <(xi + delta)^a> given m_b = <xi^b>.
void shift_moments4(const double m[N4], const int delta[3], double out[N4]);
void shift_moments3(const double m[N3], const int delta[3], double out[N3]);

// The paper's boundary fitting on the cut cells of L (ascending index), as a
// check of the exact geometry: per cell the height axis (-1: fewer than 6
// boundary points), the 6 coefficients of the quadratic height function in
// cell-centred coordinates scaled by h, and (volume, patch area, average of u
// over the region, over the patch) for the exact and the fitted region.
// Null outputs are skipped.  (fitted.cpp)
void fit_cut_cells(const LevelHost& L, const DomainSpec& dom, const FieldDesc& u, int* cell, int* axis, double* coef,
                   double* exact, double* fitted);

}  // namespace cc
