// opcount.cpp -- host program that counts the floating-point operations of
// one cell update of the step (algorithmic count: each edge solved once per
// cell and direction, no halo recomputation) by running the kernel's math
// functions on a number type that counts +, -, *, / and sqrt.  Operations on
// literal zeros and between literal constants are not counted (the compiler
// folds them).  Build: g++ -std=c++17 -O0 -o opcount opcount.cpp
#include <cstdio>
#include <cmath>
struct Cnt { long add = 0, mul = 0, div = 0, sqrt = 0; } C;
// z marks a structural zero (a literal 0 in the code): operations with it
// are folded by the compiler and not counted; c marks other literals
struct CF {
  double v; bool z, c;
  CF() : v(0), z(true), c(true) {}
  CF(double x) : v(x), z(x == 0.0), c(true) {}
  CF(double x, bool zz, bool cc) : v(x), z(zz), c(cc) {}
  explicit operator double() const { return v; }
};
inline CF mk(double v, bool z, bool c) { return CF(v, z, c); }
inline CF operator+(CF a, CF b) { if (a.z) return b; if (b.z) return a; if (!(a.c && b.c)) C.add++; return mk(a.v + b.v, false, a.c && b.c); }
inline CF operator-(CF a, CF b) { if (b.z) return a; if (a.z) return mk(-b.v, false, b.c); if (!(a.c && b.c)) C.add++; return mk(a.v - b.v, false, a.c && b.c); }
inline CF operator-(CF a) { return mk(-a.v, a.z, a.c); }
inline CF operator*(CF a, CF b) { if (a.z || b.z) return CF(); if (!(a.c && b.c)) C.mul++; return mk(a.v * b.v, false, a.c && b.c); }
inline CF operator/(CF a, CF b) { if (a.z) return CF(); if (!(a.c && b.c)) C.div++; return mk(a.v / b.v, false, a.c && b.c); }
inline CF& operator+=(CF& a, CF b) { a = a + b; return a; }
inline CF& operator-=(CF& a, CF b) { a = a - b; return a; }
inline CF& operator*=(CF& a, CF b) { a = a * b; return a; }
inline bool operator<(CF a, CF b) { return a.v < b.v; }
inline bool operator>(CF a, CF b) { return a.v > b.v; }
inline bool operator<=(CF a, CF b) { return a.v <= b.v; }
inline bool operator>=(CF a, CF b) { return a.v >= b.v; }
inline bool operator==(CF a, CF b) { return a.v == b.v; }
inline bool operator!=(CF a, CF b) { return a.v != b.v; }
inline CF sqrt(CF a) { if (!a.c) C.sqrt++; return mk(std::sqrt(a.v), a.z, a.c); }
inline CF fabs(CF a) { return mk(std::fabs(a.v), a.z, a.c); }
inline CF quot(CF a, CF b, CF) { return a / b; }
inline CF front_root(CF g, CF h, CF, CF) { return sqrt(g * h); }
inline CF frcp(CF x) { return CF(1.0) / x; }
// the kernel's reciprocal, square root and quotient helpers, counted as
// one division or square root each
inline CF recip(CF x) { return CF(1.0) / x; }
inline CF tsqrt(CF a) { return sqrt(a); }
inline CF tdiv(CF a, CF b) { return a / b; }
#include "hsgn_math.hpp"
namespace hsgn {
template <> inline CF tiny_norm<CF>() { return CF(1e-200); }
}
using namespace hsgn;
int main() {
  StepParams P; P.g = 9.81; P.a2g = 9 * 9.81; P.c2f = 0; P.eta0 = 0; P.h_star = 0.05; P.dry_tol = 1e-3; P.xi0 = 0.01; P.xi1 = 0.05; P.kappa = 0.8; P.limiter = 2; P.transverse = 2; P.splitting = 1; P.model = 0;
  auto mkcell = [&](double h, double u, double v, double b) { Cell<CF> c; double q[7] = {h, h*u, h*v, 0.01*h, 0.02*h, 0.1*h, 0.15*h}; for (int m=0;m<7;m++) c.q[m]=mk(q[m],false,false); c.b = mk(b,false,false); c.c2 = mk(9*9.81*(-b),false,false); derive(P, c); c.eta = c.h + c.b; return c; };
  Cell<CF> a = mkcell(1.0, 0.1, 0.05, -1.0), b = mkcell(1.02, 0.12, 0.04, -0.98);
  auto snap = [&](const char* what) { long t = C.add + C.mul + C.div + C.sqrt; printf("%-34s add %4ld mul %4ld div %3ld sqrt %2ld total %5ld\n", what, C.add, C.mul, C.div, C.sqrt, t); C = Cnt(); return t; };
  C = Cnt(); long total = 0;
  { CF q[7]; for (int m=0;m<7;m++) q[m]=a.q[m]; source_step(q, a.c2, mk(0.001,false,false)); } total += 2 * snap("source half step (x2 per cell)");
  { Cell<CF> c = a; derive(P, c); c.eta = c.h + c.b; } total += snap("primitives, sqrt(h), wave speed");
  Side<CF> sa, sb; side_of<0>(a, sa); side_of<0>(b, sb); C = Cnt();
  Waves<CF> W; Eig<CF> E; riemann<0>(P, sa, sb, W, E); total += 2 * snap("normal solve (x2 per cell)");
  CF d[7]; family_dots<0>(W, W, d); total += 2 * snap("neighbour dot products (x2)");
  CF F[7], am[7], ap[7]; CF dl[7], dr[7]; for (int f=0;f<7;f++){dl[f]=CF(0.5)*d[f]; dr[f]=d[f];} C = Cnt();
  correction<0>(limiter_of<CF>(2), mk(0.01,false,false), W, dl, dr, F); total += 2 * snap("limited correction (x2)");
  fluctuations<0>(W, am, ap); total += 2 * snap("fluctuations (x2)");
  CF vp[7]; CF v[7]; for (int m=0;m<7;m++) v[m]=am[m]; C = Cnt();
  trans_split<1>(E, v, 1, vp); total += 4 * snap("transverse split (x4 per cell)");
  // per cell accumulations: x: 7*(2 sub + 1 add + 1 mul + 1 sub), transverse sums, y parts
  C.add += 7 * (2 + 1 + 1 + 2 + 2 + 2 + 2 + 2 + 2 + 2); C.mul += 7 * 8;
  total += snap("update accumulation (estimate)");
  printf("TOTAL algorithmic flops per cell update: %ld\n", total);
}
