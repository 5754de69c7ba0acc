// Quadrature on boxes cut by a level set: the dimension-recursive
// height-function rule (R. Saye, SIAM J. Sci. Comput. 37 (2015) A993), used for
// the cut-cell volumes, moments and boundary-patch integrals of Sec. 2.2-2.3
// on exact obstacles: ellipsoids (quadrics) and tori (quartics, the paper's
// Problem 2).  Decisions (sign tests, height axis, bisection) follow fixed
// rules so that independent implementations agree node for node.
#pragma once
#include <vector>

namespace cc {

// phi(x) = x^T Q x + b^T x + c in e <= 3 variables (Q symmetric).
struct Quadric {
  int e = 3;
  double Q[3][3] = {};
  double b[3] = {};
  double c = 0.0;
  double eval(const double* x) const;
  void grad(const double* x, double* g) const;
  Quadric restrict_to(int k, double val) const;  // fix x_k = val, drop variable k
};

Quadric ellipsoid_quadric(const double center[3], const double axes[3], const double rot[9]);

// p(x) = sum_a c[a] x^a over exponents a of total degree <= 4 in e <= 3
// variables; c is dense with index sum_i a_i 5^(e-1-i) (entries of degree > 4
// stay 0).  Bounds on a box come from the Taylor expansion at its centre in
// the scaled variables t (x = m + w t, |t_i| <= 1): |p - d_0| <= sum_{a != 0} |d_a|.
struct Poly {
  static constexpr int kDeg = 4;
  int e = 3;
  double c[125] = {};
  double eval(const double* x) const;
  void grad(const double* x, double* g) const;
  Poly restrict_to(int k, double val) const;
  Poly deriv(int k) const;
  // value at the box centre and the bound of |p - value| on the box
  void bounds(const double* lo, const double* hi, double& v, double& spread) const;
  // coefficients a[0..4] of p along x_k at the base point xo (the other e-1
  // coordinates in ascending axis order): p = sum_j a_j x_k^j
  void line(int k, const double* xo, double a[5]) const;
};

// (|x-c|^2 + R^2 - r^2)^2 - 4 R^2 rho^2, rho the distance of x from the axis
// through `center` along the third column of rot (row-major): negative inside
// the solid torus of major radius R and minor radius r (r < R).
Poly torus_poly(const double center[3], double R, double r, const double rot[9]);

// The level set of one obstacle, positive in Omega.
struct LevelSet {
  bool poly = false;
  Quadric q;
  Poly p;
  double eval(const double* x) const { return poly ? p.eval(x) : q.eval(x); }
  void grad(const double* x, double* g) const { poly ? p.grad(x, g) : q.grad(x, g); }
  LevelSet restrict_to(int k, double val) const;
  int dim() const { return poly ? p.e : q.e; }
};

// Nodes of dimension e, row-major (P x e), weights (P).
struct NodeSet {
  int e = 0;
  std::vector<double> x;
  std::vector<double> w;
  size_t size() const { return w.size(); }
};

struct SurfaceSet {
  std::vector<double> x;  // P x 3
  std::vector<double> w;  // area element
  std::vector<double> n;  // P x 3 unit normals pointing out of {phi > 0}
};

// One line piece of a volume rule in 3 dimensions: the q-point Gauss rule on
// [a, b] along axis k at the base point xo (the other two coordinates in
// ascending axis order); node j sits at (a+b)/2 + (b-a)/2 t_j with weight
// w (b-a)/2 w_j.  A volume rule is a list of such pieces (12 times fewer
// numbers than its nodes).
struct LinePiece {
  double xo[2];
  double a, b, w;
  int k;
  int pad_;
};

constexpr int kQuadOrder = 12;     // Gauss points per piece
constexpr int kMaxDepth = 12;      // bisection limit per recursion dimension
constexpr int kPolySplitDepth = 4; // the same limit for polynomial functions in the
                                   // base splitting: a face tangent to a torus along a
                                   // circle leaves a double zero there that no box
                                   // bound separates, and bisecting along it to depth
                                   // 12 costs ~2^12 boxes; transversal zero sets of a
                                   // torus resolve by depth 1
constexpr double kTie = 1e-12;     // relative tie tolerance in axis choice
constexpr double kSlope = 4.0;     // bounded-slope test of the top-level height axis

// Volume nodes of {phi > 0} in the box and, for e == 3, surface nodes of {phi = 0}.
void region_rules(const double* lo, const double* hi, int e, const LevelSet& psi, int q,
                  NodeSet& vol, SurfaceSet* surf, int depth = 0);

// The same volume rule as line pieces (e == 3), and the same surface nodes.
void region_pieces(const double* lo, const double* hi, const LevelSet& psi, int q,
                   std::vector<LinePiece>& vol, SurfaceSet* surf);

// Gauss-Legendre nodes/weights on [-1, 1].
void gauss_legendre(int q, std::vector<double>& x, std::vector<double>& w);

}  // namespace cc
