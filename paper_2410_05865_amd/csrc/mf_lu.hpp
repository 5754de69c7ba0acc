// Nested-dissection ordering and multifrontal LU (Secs. 5.1-5.2, the
// LU-correction of Sec. 5.3 and the bottom solver), prepared for a level-by-
// level supernodal solve on the GPU.
//
// Ordering: recursive coordinate bisection of the matrix graph (pattern of
// A + A^T); the separator of a split is the set of left-side vertices adjacent to
// the right side, numbered after both halves (the recursion of the ND algorithm,
// with the slab separators of the sqrt(n)-separator proposition of Sec. 5.4).
// Factorization: per supernode (one separator or leaf), a dense front over its
// variables F and the later variables U it touches; restricted partial pivoting
// among the rows of F.  Stored per node, for the solve:
//   M (p x p): strict lower part = inverse of the unit lower factor L11,
//              upper part (with diagonal) = inverse of U11;
//   V (q x p) = L21 L11^-1,  W (p x q) = U11^-1 U12,  piv (p): pivoted row order,
//   U (q): the later variables of the front.
#pragma once
#include <array>
#include <vector>

namespace cc {

struct CSR {
  int n = 0;
  std::vector<int> ptr, col;
  std::vector<double> val;
};

struct SnNode {
  int base = 0, p = 0, q = 0;     // variables base..base+p-1; q later variables
  long long offM = 0, offV = 0, offW = 0, offU = 0, offPiv = 0;
  int height = 0;                 // 0 for leaves
  int parent = -1;
};

struct SupernodalLU {
  int n = 0;
  std::vector<int> perm;          // perm[v] = original index of variable v
  std::vector<int> iperm;         // iperm[original] = v
  std::vector<SnNode> nodes;      // postorder
  std::vector<double> Mbuf, Vbuf, Wbuf;
  std::vector<int> Ubuf, Pivbuf;
  int max_height = 0;
  long long entries() const { return (long long)(Mbuf.size() + Vbuf.size() + Wbuf.size()); }
};

// Factor A (n x n CSR) with vertex coordinates coords (grid indices) for the
// bisection; leaves hold at most `leaf` vertices.  Throws cc::Error(CC_ESINGULAR)
// if a pivot falls below pivot_tol times the largest entry of A.
void factorize(const CSR& A, const std::vector<std::array<int, 3>>& coords, int leaf, double pivot_tol,
               SupernodalLU& out);

// Host check of a factorization: solves A x = b with the stored factors (the
// same operations the device kernels perform) and returns max|A x - b| / max|b|.
double selfcheck(const CSR& A, const SupernodalLU& F, unsigned seed);

}  // namespace cc
