/*
 * Operation count of the oracle's evaluation (TEST INFRASTRUCTURE ONLY).
 *
 * The oracle's C source is compiled here a second time with its number
 * type replaced by a counting type, so the count follows exactly the steps
 * the oracle takes.  The count fixes the algorithmic work per face and per
 * cell that the roofline fractions of the benchmark divide by.  Rules:
 *
 *   - each +, -, *, /, square root and comparison of two numbers is one
 *     operation, in one of five classes (add/sub, mul, div, sqrt, cmp);
 *   - numbers that are program constants (literals, grid spacing, epsilon,
 *     time step) are "constants"; an operation on two constants is folded
 *     (free), and so are x + 0, x - 0, 0 - x, x * 0, x * (+-1), x / (+-1)
 *     and 0 / x: the structural zeros and ones of L, R and the flux
 *     directions cost nothing;
 *   - a division by a constant power of two is a multiplication;
 *   - negation and absolute value are free (operand modifiers);
 *   - an operation repeated on the same operands inside one counted unit
 *     is counted once (common subexpressions; a negated operand is the
 *     negation of the operation on the plain one), so a value is paid for
 *     once however often the oracle's plain code recomputes it;
 *   - only operations that an output of the unit or a comparison depends on
 *     are counted: a value the oracle computes and then discards (the star
 *     state of the downwind side of eq. (14), the weights of the 3-point
 *     stencils at third order) costs nothing, while a comparison, which
 *     decides what is computed, is always counted with what it compares.
 *
 * Units: one face (or_face), one piece of a face, one cell's primitive
 * recovery, one grid line of the semi-discrete operator, a whole
 * right-hand side or RK3 step.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#include <cstring>
#include <unordered_map>
#include <vector>

enum { OC_ADD, OC_MUL, OC_DIV, OC_SQRT, OC_CMP, OC_NCLASS };
enum { K_ADD, K_SUB, K_MUL, K_DIV, K_SQRT, K_NEG, K_ABS, K_LT, K_LE, K_EQ, K_NE };
enum { C_FREE = -1, C_LEAF = -2 };

struct OcNum {
  double v;
  uint32_t id; /* 0: a constant; else a node of the current unit */
  OcNum() = default;
  constexpr OcNum(double x) : v(x), id(0) {}
  constexpr OcNum(double x, uint32_t i) : v(x), id(i) {}
};

namespace {

struct Key {
  int op;
  uint32_t ia, ib;
  uint64_t ca, cb;
  bool operator==(const Key &o) const {
    return op == o.op && ia == o.ia && ib == o.ib && ca == o.ca && cb == o.cb;
  }
};
struct KeyHash {
  size_t operator()(const Key &k) const {
    uint64_t h = (uint64_t)k.op * 0x9E3779B97F4A7C15ull;
    h ^= (uint64_t)k.ia + 0x632BE59BD9B4E019ull + (h << 6) + (h >> 2);
    h ^= (uint64_t)k.ib + 0x85EBCA77C2B2AE63ull + (h << 6) + (h >> 2);
    h ^= k.ca + (h << 6) + (h >> 2);
    h ^= k.cb + (h << 6) + (h >> 2);
    return (size_t)h;
  }
};

struct Node {
  int op, cls;
  uint32_t a, b; /* operand nodes (0: a constant or none) */
};

/* The operations of one counted unit: a graph with shared subexpressions.
 * Comparisons are roots (a decision needs its operands); at the end of the
 * unit the operations reachable from the outputs or a root are counted. */
struct Graph {
  std::vector<Node> nodes;
  std::vector<uint32_t> roots;
  std::unordered_map<Key, uint32_t, KeyHash> table;
  void reset() {
    nodes.assign(1, Node{0, C_LEAF, 0, 0});
    roots.clear();
    if (table.bucket_count() > (1u << 16)) {
      std::unordered_map<Key, uint32_t, KeyHash> t;
      table.swap(t);
    } else {
      table.clear();
    }
  }
};
Graph oc;

uint64_t bits(double x) {
  uint64_t b;
  std::memcpy(&b, &x, 8);
  return b;
}
bool is_const(const OcNum &a, double c) { return a.id == 0 && a.v == c; }
bool is_pow2(double c) {
  int e;
  const double m = frexp(fabs(c), &e);
  return c != 0.0 && m == 0.5;
}
uint32_t leaf() {
  oc.nodes.push_back(Node{-1, C_LEAF, 0, 0});
  return (uint32_t)(oc.nodes.size() - 1);
}
/* The node of (op, a, b), created the first time it is evaluated. */
uint32_t node(int op, int cls, const OcNum &a, const OcNum &b) {
  Key k{op, a.id, b.id, a.id ? 0 : bits(a.v), b.id ? 0 : bits(b.v)};
  auto it = oc.table.find(k);
  if (it != oc.table.end()) return it->second;
  oc.nodes.push_back(Node{op, cls, a.id, b.id});
  const uint32_t id = (uint32_t)(oc.nodes.size() - 1);
  oc.table.emplace(k, id);
  if (cls == OC_CMP) oc.roots.push_back(id);
  return id;
}
/* Commutative operations see their operands in one canonical order. */
void order(const OcNum *&a, const OcNum *&b) {
  if (a->id > b->id || (a->id == b->id && bits(a->v) > bits(b->v))) {
    const OcNum *t = a;
    a = b;
    b = t;
  }
}
bool is_neg(const OcNum &a) { return a.id && oc.nodes[a.id].op == K_NEG; }
OcNum src(const OcNum &a) { return OcNum(-a.v, oc.nodes[a.id].a); }

OcNum neg(const OcNum &a) {
  if (!a.id) return OcNum(-a.v);
  if (is_neg(a)) return src(a);
  return OcNum(-a.v, node(K_NEG, C_FREE, a, OcNum(0.0)));
}

/* Counts of the operations that the outputs or a decision depend on; the
 * values in stop (if any) are taken as given, like inputs. */
void count(const OcNum *out, long nout, long *counts, const OcNum *stop = nullptr,
           long nstop = 0) {
  std::vector<char> seen(oc.nodes.size(), 0);
  for (long i = 0; i < nstop; i++) seen[stop[i].id] = 1;
  std::vector<uint32_t> stack(oc.roots);
  for (long i = 0; i < nout; i++)
    if (out[i].id) stack.push_back(out[i].id);
  for (int c = 0; c < OC_NCLASS; c++) counts[c] = 0;
  while (!stack.empty()) {
    const uint32_t id = stack.back();
    stack.pop_back();
    if (!id || seen[id]) continue;
    seen[id] = 1;
    const Node &n = oc.nodes[id];
    if (n.cls >= 0) counts[n.cls]++;
    stack.push_back(n.a);
    stack.push_back(n.b);
  }
}

}  // namespace

OcNum operator-(const OcNum &a) { return neg(a); }
OcNum operator-(const OcNum &x, const OcNum &y);

OcNum operator+(const OcNum &x, const OcNum &y) {
  const double v = x.v + y.v;
  if (!x.id && !y.id) return OcNum(v);
  if (is_const(x, 0.0)) return y;
  if (is_const(y, 0.0)) return x;
  if (is_neg(y)) return x - src(y);
  if (is_neg(x)) return y - src(x);
  const OcNum *a = &x, *b = &y;
  order(a, b);
  return OcNum(v, node(K_ADD, OC_ADD, *a, *b));
}
OcNum operator-(const OcNum &x, const OcNum &y) {
  const double v = x.v - y.v;
  if (!x.id && !y.id) return OcNum(v);
  if (is_const(y, 0.0)) return x;
  if (is_const(x, 0.0)) return neg(y);
  if (is_neg(y)) return x + src(y);
  if (is_neg(x)) return neg(src(x) + y);
  return OcNum(v, node(K_SUB, OC_ADD, x, y));
}
OcNum operator*(const OcNum &x, const OcNum &y) {
  const double v = x.v * y.v;
  if (!x.id && !y.id) return OcNum(v);
  if (is_const(x, 0.0) || is_const(y, 0.0)) return OcNum(v);
  if (is_const(x, 1.0)) return y;
  if (is_const(y, 1.0)) return x;
  if ((!x.id && x.v < 0.0) || is_neg(x)) return neg(neg(x) * y);
  if ((!y.id && y.v < 0.0) || is_neg(y)) return neg(x * neg(y));
  const OcNum *a = &x, *b = &y;
  order(a, b);
  return OcNum(v, node(K_MUL, OC_MUL, *a, *b));
}
OcNum operator/(const OcNum &x, const OcNum &y) {
  const double v = x.v / y.v;
  if (!x.id && !y.id) return OcNum(v);
  if (is_const(x, 0.0)) return OcNum(v);
  if (is_const(y, 1.0)) return x;
  if ((!x.id && x.v < 0.0) || is_neg(x)) return neg(neg(x) / y);
  if ((!y.id && y.v < 0.0) || is_neg(y)) return neg(x / neg(y));
  const int cls = (!y.id && is_pow2(y.v)) ? OC_MUL : OC_DIV;
  return OcNum(v, node(K_DIV, cls, x, y));
}
OcNum &operator+=(OcNum &a, const OcNum &b) { return a = a + b; }
OcNum &operator-=(OcNum &a, const OcNum &b) { return a = a - b; }
OcNum &operator*=(OcNum &a, const OcNum &b) { return a = a * b; }
OcNum &operator/=(OcNum &a, const OcNum &b) { return a = a / b; }

static bool cmp(int op, const OcNum &x, const OcNum &y, bool r, bool sym) {
  if (x.id || y.id) {
    const OcNum *a = &x, *b = &y;
    if (sym) order(a, b);
    node(op, OC_CMP, *a, *b);
  }
  return r;
}
bool operator<(const OcNum &a, const OcNum &b) { return cmp(K_LT, a, b, a.v < b.v, false); }
bool operator>(const OcNum &a, const OcNum &b) { return cmp(K_LT, b, a, a.v > b.v, false); }
bool operator<=(const OcNum &a, const OcNum &b) { return cmp(K_LE, a, b, a.v <= b.v, false); }
bool operator>=(const OcNum &a, const OcNum &b) { return cmp(K_LE, b, a, a.v >= b.v, false); }
bool operator==(const OcNum &a, const OcNum &b) { return cmp(K_EQ, a, b, a.v == b.v, true); }
bool operator!=(const OcNum &a, const OcNum &b) { return cmp(K_NE, a, b, a.v != b.v, true); }

OcNum sqrt(const OcNum &a) {
  const double v = std::sqrt(a.v);
  if (!a.id) return OcNum(v);
  return OcNum(v, node(K_SQRT, OC_SQRT, a, OcNum(0.0)));
}
OcNum fabs(const OcNum &a) {
  const double v = std::fabs(a.v);
  if (!a.id) return OcNum(v);
  if (is_neg(a)) return fabs(src(a));
  return OcNum(v, node(K_ABS, C_FREE, a, OcNum(0.0)));
}
bool isfinite(const OcNum &a) { return std::isfinite(a.v); }

/* The oracle itself, on the counting type. */
#define double OcNum
#include "oracle.c"
#undef double

/* ------------------------------------------------------------------------ */
/* Entry points (plain doubles in, counts out)                               */
/* ------------------------------------------------------------------------ */

#define OC_API extern "C" __attribute__((visibility("default")))

namespace {

/* Inputs are data, never constants: each value is a leaf of its own. */
OcNum *lift(const double *x, long n) {
  OcNum *y = (OcNum *)malloc(sizeof(OcNum) * (size_t)(n > 0 ? n : 1));
  for (long i = 0; i < n; i++) y[i] = OcNum(x[i], leaf());
  return y;
}
or_grid grid_of(int ndim, const long *n, const double *dx, const int *bc_lo,
                const int *bc_hi) {
  or_grid g;
  memset(&g, 0, sizeof(g));
  g.ndim = ndim;
  for (int a = 0; a < 3; a++) {
    g.n[a] = a < ndim ? n[a] : 1;
    g.dx[a] = OcNum(a < ndim ? dx[a] : 1.0);
    g.bc_lo[a] = a < ndim ? bc_lo[a] : 0;
    g.bc_hi[a] = a < ndim ? bc_hi[a] : 0;
  }
  return g;
}
or_opts opts_of(int weights, int mood, double eps) {
  or_opts o;
  o.weights = weights;
  o.mood = mood;
  o.eps = OcNum(eps);
  o.cfl = OcNum(0.0);
  return o;
}
/* One face on fresh leaves; counts over its flux and u^HLLC. */
void face_count(int nt, const double *q6, const or_opts *o, long *counts, int *ord) {
  const int nc = 5 + nt;
  oc.reset();
  OcNum *q = lift(q6, 6L * nc);
  OcNum ql[OR_MAXNC], qr[OR_MAXNC], out[OR_MAXNC + 1];
  or_face(nt, q, o, ql, qr, ord, out, out + nc);
  count(out, nc + 1, counts);
  free(q);
}

}  // namespace

/* One face from its six primitive cell states (face order, 6 x nc). */
OC_API int oc_face(int nt, const double *q6, int weights, int mood, double eps,
                   long *counts, int *order_lr) {
  if (nt < 0 || nt > 2 || !q6 || !counts) return OR_ERR_ARG;
  const or_opts o = opts_of(weights, mood, eps);
  int ord[2];
  face_count(nt, q6, &o, counts, ord);
  if (order_lr) {
    order_lr[0] = ord[0];
    order_lr[1] = ord[1];
  }
  return OR_OK;
}

/* Pieces of a face, for checking the count against hand counts:
 * 0 WENO-IS value (eq. (19)) from v[5] at order `order`;
 * 1 face matrices at the average of cells 2 and 3 of q6 and the projection
 *   of the six cells (eqs. (11), (12));
 * 2 HLLC flux and u^HLLC (eqs. (14)-(18)) from ql = x[0..nc), qr = x[nc..2nc);
 * 3 positivity test of a face state x[0..nc). */
OC_API int oc_piece(int kind, int nt, const double *x, int weights, double eps,
                    int order, long *counts) {
  if (nt < 0 || nt > 2 || !x || !counts) return OR_ERR_ARG;
  const int nc = 5 + nt;
  oc.reset();
  if (kind == 0) {
    OcNum *v = lift(x, 5);
    OcNum q = or_weno_is(v, weights, OcNum(eps), order);
    count(&q, 1, counts);
    free(v);
  } else if (kind == 1) {
    OcNum *q6 = lift(x, 6L * nc);
    OcNum qbar[OR_MAXNC], L[OR_MAXNC * OR_MAXNC], R[OR_MAXNC * OR_MAXNC];
    OcNum w[6 * OR_MAXNC];
    for (int k = 0; k < nc; k++) qbar[k] = 0.5 * (q6[2 * nc + k] + q6[3 * nc + k]);
    or_eigen(nt, qbar, L, R);
    for (int j = 0; j < 6; j++) matvec(nc, L, q6 + j * nc, w + j * nc);
    count(w, 6L * nc, counts);
    free(q6);
  } else if (kind == 2) {
    OcNum *q = lift(x, 2L * nc);
    OcNum out[OR_MAXNC + 1];
    or_hllc(nt, q, q + nc, out, out + nc);
    count(out, nc + 1, counts);
    free(q);
  } else if (kind == 3) {
    OcNum *q = lift(x, nc);
    (void)or_pos(nt, q);
    count(nullptr, 0, counts);
    free(q);
  } else {
    return OR_ERR_ARG;
  }
  return OR_OK;
}

/* Primitive recovery of one cell (u: its nc conservative values). */
OC_API int oc_prim(int ndim, const double *u, int d, long *counts) {
  if (ndim < 1 || ndim > 3 || d < 0 || d >= ndim || !u || !counts) return OR_ERR_ARG;
  oc.reset();
  OcNum *U = lift(u, 4 + ndim);
  OcNum q[OR_MAXNC];
  cell_prim(ndim, 1, U, 0, d, q);
  count(q, 4 + ndim, counts);
  free(U);
  return OR_OK;
}

/* One grid line of direction d (the line through cell `base`, whose index
 * along d is 0).  total: the line's whole evaluation (primitive recovery,
 * faces, flux differences and sources, and for d > 0 the sum with the
 * earlier axes' terms); faces: its faces counted one by one, each alone;
 * assembly: what the flux differences, sources and sums add to the faces
 * and primitive states (found by evaluating the faces again in the line's
 * graph, which must only meet operations it already holds). */
OC_API int oc_line(int ndim, const long *n, const double *dx, const int *bc_lo,
                   const int *bc_hi, int weights, int mood, double eps,
                   const double *U, int d, long base, long *total, long *faces,
                   long *assembly) {
  if (ndim < 1 || ndim > 3 || d < 0 || d >= ndim || !U || !total || !faces || !assembly)
    return OR_ERR_ARG;
  const or_grid g = grid_of(ndim, n, dx, bc_lo, bc_hi);
  if (!check_grid(&g)) return OR_ERR_ARG;
  const or_opts o = opts_of(weights, mood, eps);
  const long nce = ncells(&g), nc = 4 + ndim, nd = g.n[d];
  long stride = 1, o3 = 0, o1 = 0;
  for (int a = 0; a < d; a++) stride *= g.n[a];
  if (base < 0 || base >= nce || (base / stride) % nd != 0) return OR_ERR_ARG;
  const int nt = ndim - 1, ncf = 5 + nt;
  /* whole line, one graph; outputs are the line's cells of dU/dt */
  oc.reset();
  OcNum *Ul = lift(U, nc * nce);
  OcNum *dU = lift(U, nc * nce); /* partial sums of earlier axes */
  line_rhs(&g, &o, Ul, dU, d, base, stride, &o3, &o1);
  OcNum *out = (OcNum *)malloc(sizeof(OcNum) * (size_t)(nd * nc));
  for (long i = 0; i < nd; i++)
    for (long k = 0; k < nc; k++) out[i * nc + k] = dU[k * nce + base + i * stride];
  count(out, nd * nc, total);
  free(out);
  /* the faces again, inside the same graph */
  const size_t before = oc.nodes.size();
  OcNum *ext = (OcNum *)malloc(sizeof(OcNum) * (size_t)(nd + 6) * ncf);
  OcNum *fo = (OcNum *)malloc(sizeof(OcNum) * (size_t)(nd + 1) * (ncf + 1));
  for (long l = -3; l < nd + 3; l++) {
    int flip;
    const long c = bc_map(l, nd, g.bc_lo[d], g.bc_hi[d], &flip);
    OcNum *q = ext + (l + 3) * ncf;
    cell_prim(ndim, nce, Ul, base + c * stride, d, q);
    if (flip) q[1] = -q[1];
  }
  for (long f = 0; f <= nd; f++) {
    OcNum ql[OR_MAXNC], qr[OR_MAXNC];
    int ord[2];
    OcNum *F = fo + f * (ncf + 1);
    or_face(nt, ext + f * ncf, &o, ql, qr, ord, F, F + ncf);
  }
  const bool same = oc.nodes.size() == before;
  long fl[OC_NCLASS];
  count(fo, (nd + 1) * (ncf + 1), fl);
  for (int c = 0; c < OC_NCLASS; c++) assembly[c] = total[c] - fl[c];
  free(Ul);
  free(dU);
  free(fo);
  /* the same faces, each alone */
  double *raw = (double *)malloc(sizeof(double) * (size_t)(nd + 6) * ncf);
  for (long k = 0; k < (nd + 6) * ncf; k++) raw[k] = ext[k].v;
  free(ext);
  long fc[OC_NCLASS];
  int ord[2];
  for (int c = 0; c < OC_NCLASS; c++) faces[c] = 0;
  for (long f = 0; f <= nd; f++) {
    face_count(nt, raw + f * ncf, &o, fc, ord);
    for (int c = 0; c < OC_NCLASS; c++) faces[c] += fc[c];
  }
  free(raw);
  return same ? OR_OK : OR_ERR_NONPHYSICAL;
}

/* A whole right-hand side (rk3 = 0) or RK3 step (rk3 = 1) in one graph;
 * outputs are every value of dU/dt or of the new state.  For a step,
 * update receives what the three stage updates add to the three right-hand
 * sides (found by evaluating the stages again inside the step's graph,
 * which must only meet operations it already holds). */
OC_API int oc_eval(int ndim, const long *n, const double *dx, const int *bc_lo,
                   const int *bc_hi, int weights, int mood, double eps,
                   const double *U, int rk3, double dt, long *counts, long *update) {
  if (ndim < 1 || ndim > 3 || !U || !counts || (rk3 && !update)) return OR_ERR_ARG;
  const or_grid g = grid_of(ndim, n, dx, bc_lo, bc_hi);
  if (!check_grid(&g)) return OR_ERR_ARG;
  const or_opts o = opts_of(weights, mood, eps);
  const long m = (4 + ndim) * ncells(&g);
  oc.reset();
  OcNum *Ul = lift(U, m);
  OcNum *out = (OcNum *)malloc(sizeof(OcNum) * (size_t)m * 3);
  or_stats st;
  memset(&st, 0, sizeof(st));
  int s;
  if (!rk3) {
    s = or_rhs(&g, &o, Ul, out, &st);
    count(out, m, counts);
  } else {
    OcNum *U0 = (OcNum *)malloc(sizeof(OcNum) * (size_t)m);
    memcpy(U0, Ul, sizeof(OcNum) * (size_t)m);
    s = or_rk3_step(&g, &o, Ul, OcNum(dt), &st);
    count(Ul, m, counts);
    /* the stages again: the three right-hand sides */
    const size_t before = oc.nodes.size();
    const OcNum h = OcNum(dt);
    OcNum *Us = (OcNum *)malloc(sizeof(OcNum) * (size_t)m * 2);
    or_rhs(&g, &o, U0, out, &st);
    for (long i = 0; i < m; i++) Us[i] = U0[i] + h * out[i];
    or_rhs(&g, &o, Us, out + m, &st);
    for (long i = 0; i < m; i++) Us[m + i] = 0.75 * U0[i] + 0.25 * (Us[i] + h * out[m + i]);
    or_rhs(&g, &o, Us + m, out + 2 * m, &st);
    if (oc.nodes.size() != before) s = OR_ERR_NONPHYSICAL;
    long r[OC_NCLASS];
    count(out, 3 * m, r, Us, 2 * m); /* the stage states themselves excluded */
    for (int c = 0; c < OC_NCLASS; c++) update[c] = counts[c] - r[c];
    free(Us);
    free(U0);
  }
  free(Ul);
  free(out);
  return s;
}
