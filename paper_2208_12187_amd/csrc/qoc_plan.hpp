// Choice of the scaling exponent s and the Taylor degrees (q for exp, qb for
// its Frechet block) of one slice, shared by the plan kernel and the host.
//
// theta = dt (|H0|_1 + sum_j |u[j][k]| |Hc[j]|_1) bounds |A_k|_1 by the
// triangle inequality (A_k = -i dt H_k), and |A^n| <= |A|^n in the 1-norm.
// With r = theta / 2^s:
//  * exp: the Taylor remainder after degree q is at most
//    r^(q+1)/(q+1)! * 1/(1 - r/(q+2)) (geometric bound on the tail ratios);
//    q is the least degree for which this is at most the unit roundoff ur.
//  * Frechet block exp([[X, E], [0, X]]): its top-right block is linear in E
//    and the degree-n term of the series contributes n X^(n-1)-type products,
//    so the remainder after degree qb is at most
//    |E| r^qb/qb! * 1/(1 - r/(qb+1)); qb (>= 2) is the least degree for which
//    the factor of |E| is at most ur.
// Among s in [s0, s0 + 6], s0 = least s >= 0 with r <= 1, the value that
// minimises the number of complex d x d products of the path is taken:
//    exp:       (q - 1) + s    (Horner; expm_products(q) + s where the expm
//                                 runs Paterson-Stockmeyer: FP32 at D = 128)
//    gradient:  + frechet_products(qb) + 3 s   (block polynomial, squarings)
// (where the adjoint reuses the expm's X^2 it saves one product for every s
// alike, so the choice does not depend on that).
#pragma once

#include <math.h>

namespace qoc {

struct SlicePlan {
  int s, q, qb;
};

#if defined(__HIPCC__)
#define QOC_HD __host__ __device__
#else
#define QOC_HD
#endif

QOC_HD inline int taylor_degree(double r, double ur) {
  int q = 1;
  double t = r * r * 0.5;  // r^(q+1)/(q+1)!
  while (q < 30 && t / (1.0 - r / (q + 2)) > ur) {
    ++q;
    t *= r / (q + 1);
  }
  return q;
}

QOC_HD inline int frechet_degree(double r, double ur) {
  int qb = 2;
  double t = r * r * 0.5;  // r^qb/qb!
  while (qb < 31 && t / (1.0 - r / (qb + 1)) > ur) {
    ++qb;
    t *= r / qb;
  }
  return qb;
}

QOC_HD inline double inv_factorial(int n) {
  double f = 1.0;
  for (int i = 2; i <= n; ++i) f /= i;
  return f;
}

// Complex d x d products of the degree-q Taylor polynomial in delta form by
// Paterson-Stockmeyer with X^2 as the step: one for X^2, one per digit that
// holds a matrix below the top one (floor((q - 3) / 2) of them) and one for
// the last step (q >= 3); X + X^2 / 2 at q = 2.
QOC_HD inline int expm_products(int q) { return q < 2 ? 0 : (q == 2 ? 1 : 2 + (q - 3) / 2); }

// Complex d x d products of the degree-qb Taylor polynomial of the block
// [[X, E], [0, X]] by Paterson-Stockmeyer with the block's square as the
// step: three for the square, three per Horner step in the square that has a
// matrix digit (floor((qb - 3) / 2) of them), two for the last step's top
// right block (the top left one is counted with the squarings).
QOC_HD inline int frechet_products(int qb) { return 5 + 3 * (qb > 3 ? (qb - 3) / 2 : 0); }

QOC_HD inline int plan_cost(int s, int q, int qb, bool grad, bool ps_expm) {
  int cost = (ps_expm ? expm_products(q) : q - 1) + s;
  if (grad) cost += frechet_products(qb) + 3 * s;
  return cost;
}

QOC_HD inline SlicePlan choose_plan(double theta, double ur, bool grad, bool ps_expm = false) {
  int s0 = 0;
  while (ldexp(theta, -s0) > 1.0 && s0 < 60) ++s0;
  SlicePlan best = {s0, 1, 2};
  int best_cost = 1 << 30;
  for (int s = s0; s <= s0 + 6; ++s) {
    double r = ldexp(theta, -s);
    int q = taylor_degree(r, ur);
    int qb = frechet_degree(r, ur);
    int c = plan_cost(s, q, qb, grad, ps_expm);
    if (c < best_cost) {
      best_cost = c;
      best.s = s;
      best.q = q;
      best.qb = qb;
    }
  }
  return best;
}

QOC_HD inline int pack_plan(SlicePlan p) { return p.s | (p.q << 8) | (p.qb << 16); }

}  // namespace qoc
