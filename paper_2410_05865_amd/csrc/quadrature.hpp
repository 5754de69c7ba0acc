// Quadrature on boxes cut by a quadratic level set: the dimension-recursive
// height-function rule (R. Saye, SIAM J. Sci. Comput. 37 (2015) A993), used for
// the cut-cell volumes, moments and boundary-patch integrals of Sec. 2.2-2.3
// on exact ellipsoids.  Decisions (sign tests, height axis, bisection) follow
// fixed rules so that independent implementations agree node for node.
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

constexpr int kQuadOrder = 12;     // Gauss points per piece
constexpr int kMaxDepth = 12;      // bisection limit per recursion dimension
constexpr double kTie = 1e-12;     // relative tie tolerance in axis choice
constexpr double kSlope = 4.0;     // bounded-slope test of the top-level height axis

// Volume nodes of {phi > 0} in the box and, for e == 3, surface nodes of {phi = 0}.
void region_rules(const double* lo, const double* hi, int e, const Quadric& psi, int q,
                  NodeSet& vol, SurfaceSet* surf, int depth = 0);

// Gauss-Legendre nodes/weights on [-1, 1].
void gauss_legendre(int q, std::vector<double>& x, std::vector<double>& w);

}  // namespace cc
