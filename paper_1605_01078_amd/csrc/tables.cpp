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
  std::vector<Product> t;
  for (const QProduct& qp : kOneLevel) {
    Product p;
    for (int s = 0; s < qp.na; ++s) p.a.push_back({qp.a[s].q >> 1, qp.a[s].q & 1, qp.a[s].sign});
    for (int s = 0; s < qp.nb; ++s) p.b.push_back({qp.b[s].q >> 1, qp.b[s].q & 1, qp.b[s].sign});
    for (int s = 0; s < qp.nc; ++s) p.c.push_back({qp.c[s].q >> 1, qp.c[s].q & 1, qp.c[s].sign});
    t.push_back(p);
  }
  return t;
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
