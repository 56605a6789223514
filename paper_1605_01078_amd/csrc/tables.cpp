// Strassen operation tables on the library side.
//
// One level: the seven operations of Fig. "All operations for one-level Strassen" (Sec. 3.1).
// L levels (Sec. 3.5): product 7^(L-1)*r + s applies outer row r of the one-level table to the
// 2x2 grid of 2^(L-1)-blocks and row s of the (L-1)-level table inside them.  Block indices
// combine as 2^(L-1)*outer + inner; coefficients multiply.  Terms are kept inner-term-major,
// the order in which the paper lists the two-level operand sums.
#include "plan.h"

namespace smx {

namespace {

std::vector<Product> one_level() {
  // {A terms}, {B terms}, {C updates}; each term is {row block, col block, sign}.
  return {
      // M0 = (A00 + A11)(B00 + B11); C00 += M0; C11 += M0
      {{{0, 0, 1}, {1, 1, 1}}, {{0, 0, 1}, {1, 1, 1}}, {{0, 0, 1}, {1, 1, 1}}},
      // M1 = (A10 + A11) B00; C10 += M1; C11 -= M1
      {{{1, 0, 1}, {1, 1, 1}}, {{0, 0, 1}}, {{1, 0, 1}, {1, 1, -1}}},
      // M2 = A00 (B01 - B11); C01 += M2; C11 += M2
      {{{0, 0, 1}}, {{0, 1, 1}, {1, 1, -1}}, {{0, 1, 1}, {1, 1, 1}}},
      // M3 = A11 (B10 - B00); C00 += M3; C10 += M3
      {{{1, 1, 1}}, {{1, 0, 1}, {0, 0, -1}}, {{0, 0, 1}, {1, 0, 1}}},
      // M4 = (A00 + A01) B11; C01 += M4; C00 -= M4
      {{{0, 0, 1}, {0, 1, 1}}, {{1, 1, 1}}, {{0, 1, 1}, {0, 0, -1}}},
      // M5 = (A10 - A00)(B00 + B01); C11 += M5
      {{{1, 0, 1}, {0, 0, -1}}, {{0, 0, 1}, {0, 1, 1}}, {{1, 1, 1}}},
      // M6 = (A01 - A11)(B10 + B11); C00 += M6
      {{{0, 1, 1}, {1, 1, -1}}, {{1, 0, 1}, {1, 1, 1}}, {{0, 0, 1}}},
  };
}

std::vector<Term> kron(const std::vector<Term>& outer, const std::vector<Term>& inner, int q_in) {
  std::vector<Term> out;
  for (const Term& ti : inner)
    for (const Term& to : outer)
      out.push_back({q_in * to.row + ti.row, q_in * to.col + ti.col, to.sign * ti.sign});
  return out;
}

}  // namespace

std::vector<Product> build_table(int levels) {
  if (levels <= 0) return {{{{0, 0, 1}}, {{0, 0, 1}}, {{0, 0, 1}}}};
  const std::vector<Product> base = one_level();
  std::vector<Product> t = base;
  for (int lev = 2; lev <= levels; ++lev) {
    const int q_in = 1 << (lev - 1);
    std::vector<Product> next;
    next.reserve(t.size() * 7);
    for (const Product& o : base)
      for (const Product& i : t)
        next.push_back({kron(o.a, i.a, q_in), kron(o.b, i.b, q_in), kron(o.c, i.c, q_in)});
    t.swap(next);
  }
  return t;
}

}  // namespace smx
