/*
 * ORACLE -- test infrastructure only (see oracle.h).
 *
 * Every quantity is computed per event from its plain definition in FP64 and
 * summed with Neumaier's compensated summation:
 *   - the PDFs of the catalogue, each normalised on its dimensions' ranges
 *     (Gaussian and exponential: Eq. 2; P-wave angular density: Eq. 4;
 *     Chebyshev series; products; sums with a fraction);
 *   - ln P and, by the chain rule through the model tree, dP/dtheta and
 *     d2P/dtheta2, giving the NLL (Eq. 1), its gradient and its Hessian;
 *   - a BFGS minimisation (the variable-metric method named for Migrad,
 *     Sec. 2.1) and the inverse Hessian at the minimum as covariance
 *     (the HESSE step of the benchmark protocol, Sec. 3.1).
 * No blocking, fusion or reordering beyond those definitions.
 */
#include "oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

#define NP ORC_MAXP

typedef struct {
  double v;
  double g[NP];
  double h[NP * NP];
} val_t;

/* ------------------------------------------------------------------ */
/* model set-up                                                        */
/* ------------------------------------------------------------------ */

int orc_model_init(orc_model* m, int ndim, const double* lo, const double* hi,
                   int nnode, const int* nodes18, int root, int npar) {
  memset(m, 0, sizeof(*m));
  if (ndim < 1 || ndim > ORC_MAXD || nnode < 1 || nnode > ORC_MAXN ||
      npar < 0 || npar > ORC_MAXP || root < 0 || root >= nnode)
    return -1;
  m->ndim = ndim;
  for (int d = 0; d < ndim; ++d) {
    m->lo[d] = lo[d];
    m->hi[d] = hi[d];
    if (!(hi[d] > lo[d])) return -2;
  }
  m->nnode = nnode;
  for (int i = 0; i < nnode; ++i) {
    const int* r = nodes18 + 18 * i;
    orc_node* nd = &m->node[i];
    nd->kind = r[0];
    for (int k = 0; k < 3; ++k) nd->dim[k] = r[1 + k];
    nd->npar = r[4];
    for (int k = 0; k < 8; ++k) nd->par[k] = r[5 + k];
    nd->nchild = r[13];
    for (int k = 0; k < 4; ++k) nd->child[k] = r[14 + k];
    if (nd->npar < 0 || nd->npar > 8 || nd->nchild < 0 || nd->nchild > 4)
      return -3;
    for (int k = 0; k < nd->npar; ++k)
      if (nd->par[k] < 0 || nd->par[k] >= npar) return -4;
    for (int k = 0; k < nd->nchild; ++k)
      if (nd->child[k] < 0 || nd->child[k] >= nnode || nd->child[k] == i)
        return -5;
  }
  m->root = root;
  m->npar = npar;
  return 0;
}

/* ------------------------------------------------------------------ */
/* leaves                                                              */
/* ------------------------------------------------------------------ */

static void clear_val(val_t* o, int order, int np) {
  o->v = 0.0;
  if (order >= 1) memset(o->g, 0, sizeof(double) * np);
  if (order >= 2) memset(o->h, 0, sizeof(double) * np * np);
}

/* Fills g = v * dl and h = v * (dl dl^T + hl) for a leaf whose log-density
 * derivatives with respect to its k parameters are dl[k] and hl[k][k]. */
static void leaf_from_log(val_t* o, int order, int np, double v, int k,
                          const int* idx, const double* dl, const double* hl) {
  o->v = v;
  if (order >= 1)
    for (int a = 0; a < k; ++a) o->g[idx[a]] += v * dl[a];
  if (order >= 2)
    for (int a = 0; a < k; ++a)
      for (int b = 0; b < k; ++b)
        o->h[idx[a] * np + idx[b]] += v * (dl[a] * dl[b] + hl[a * k + b]);
}

/* Phi(zb) - Phi(za) for za < zb, with erfc where both share a sign. */
static double phi_diff(double za, double zb) {
  const double r2 = sqrt(2.0);
  if (za >= 0.0) return 0.5 * (erfc(za / r2) - erfc(zb / r2));
  if (zb <= 0.0) return 0.5 * (erfc(-zb / r2) - erfc(-za / r2));
  return 1.0 - 0.5 * erfc(zb / r2) - 0.5 * erfc(-za / r2);
}

/* Gaussian normalised on [a, b] (Eq. 2): exp(-z^2/2) / (sigma sqrt(2 pi) D),
 * z = (x - mu)/sigma, D = Phi(zb) - Phi(za). */
static void leaf_gauss(const orc_model* m, const orc_node* nd, const double* xe,
                       const double* th, int order, val_t* o) {
  int np = m->npar, d = nd->dim[0];
  double x = xe[d], a = m->lo[d], b = m->hi[d];
  double mu = th[nd->par[0]], sg = th[nd->par[1]];
  if (!(sg > 0.0)) {
    o->v = NAN;
    return;
  }
  double z = (x - mu) / sg, za = (a - mu) / sg, zb = (b - mu) / sg;
  double D = phi_diff(za, zb);
  double v = exp(-0.5 * z * z) / (sg * sqrt(2.0 * M_PI) * D);
  if (order == 0) {
    o->v = v;
    return;
  }
  double pa = exp(-0.5 * za * za) / sqrt(2.0 * M_PI);
  double pb = exp(-0.5 * zb * zb) / sqrt(2.0 * M_PI);
  /* derivatives of D with respect to mu and sigma */
  double Dm = (pa - pb) / sg;
  double Ds = (za * pa - zb * pb) / sg;
  double Dmm = (za * pa - zb * pb) / (sg * sg);
  double Dms = (-(pa - pb) + za * za * pa - zb * zb * pb) / (sg * sg);
  double Dss = (-2.0 * za * pa + za * za * za * pa + 2.0 * zb * pb -
                zb * zb * zb * pb) / (sg * sg);
  double dl[2], hl[4];
  dl[0] = z / sg - Dm / D;
  dl[1] = z * z / sg - 1.0 / sg - Ds / D;
  hl[0] = -1.0 / (sg * sg) - (Dmm / D - Dm * Dm / (D * D));
  hl[1] = -2.0 * z / (sg * sg) - (Dms / D - Dm * Ds / (D * D));
  hl[2] = hl[1];
  hl[3] = -3.0 * z * z / (sg * sg) + 1.0 / (sg * sg) - (Dss / D - Ds * Ds / (D * D));
  int idx[2] = {nd->par[0], nd->par[1]};
  leaf_from_log(o, order, np, v, 2, idx, dl, hl);
}

/* h(z) = 1/(1 - e^{-z}) - 1/z and its derivative; series near z = 0. */
static double exp_h(double z) {
  if (fabs(z) < 0.05) {
    double z2 = z * z;
    return 0.5 + z / 12.0 - z * z2 / 720.0 + z * z2 * z2 / 30240.0 -
           z * z2 * z2 * z2 / 1209600.0;
  }
  return -1.0 / expm1(-z) - 1.0 / z;
}
static double exp_hp(double z) {
  if (fabs(z) < 0.05) {
    double z2 = z * z;
    return 1.0 / 12.0 - z2 / 240.0 + z2 * z2 / 6048.0 - z2 * z2 * z2 / 172800.0;
  }
  double em = expm1(-z);
  return 1.0 / (z * z) - exp(-z) / (em * em);
}

/* Exponential normalised on [a, b] (Eq. 2): e^{lambda x} / N,
 * N = (e^{lambda b} - e^{lambda a}) / lambda, or b - a at lambda = 0.
 * Written with expm1 so that small |lambda| keeps full precision.
 * d ln p / d lambda = x - E[x], d2 ln p / d lambda2 = -Var[x]. */
static void leaf_exp(const orc_model* m, const orc_node* nd, const double* xe,
                     const double* th, int order, val_t* o) {
  int np = m->npar, d = nd->dim[0];
  double x = xe[d], a = m->lo[d], b = m->hi[d], L = b - a;
  double lam = th[nd->par[0]];
  double v, ex, var;
  if (lam == 0.0) {
    v = 1.0 / L;
    ex = a + 0.5 * L;
    var = L * L / 12.0;
  } else {
    double z = lam * L;
    v = lam * exp(lam * (x - a)) / expm1(z);
    ex = a + L * exp_h(z);
    var = L * L * exp_hp(z);
  }
  if (order == 0) {
    o->v = v;
    return;
  }
  double dl = x - ex, hl = -var;
  int idx = nd->par[0];
  leaf_from_log(o, order, np, v, 1, &idx, &dl, &hl);
}

/* Chebyshev series on [a, b]: (1 + sum_j c_j T_j(u)) / N_C,
 * u = (2x - a - b)/(b - a), N_C = (b-a)/2 * (2 + sum_{j even} c_j 2/(1-j^2)). */
static void leaf_cheb(const orc_model* m, const orc_node* nd, const double* xe,
                      const double* th, int order, val_t* o) {
  int np = m->npar, d = nd->dim[0], k = nd->npar;
  double x = xe[d], a = m->lo[d], b = m->hi[d];
  double u = (2.0 * x - a - b) / (b - a);
  double T[9], J[9];
  T[0] = 1.0;
  T[1] = u;
  for (int j = 2; j <= k; ++j) T[j] = 2.0 * u * T[j - 1] - T[j - 2];
  double U = 1.0, N = b - a;
  for (int j = 1; j <= k; ++j) {
    J[j] = (j % 2 == 0) ? 0.5 * (b - a) * 2.0 / (1.0 - (double)(j * j)) : 0.0;
    double c = th[nd->par[j - 1]];
    U += c * T[j];
    N += c * J[j];
  }
  double v = U / N;
  o->v = v;
  if (order >= 1)
    for (int j = 1; j <= k; ++j)
      o->g[nd->par[j - 1]] += T[j] / N - U * J[j] / (N * N);
  if (order >= 2)
    for (int i = 1; i <= k; ++i)
      for (int j = 1; j <= k; ++j)
        o->h[nd->par[i - 1] * np + nd->par[j - 1]] +=
            -(T[i] * J[j] + T[j] * J[i]) / (N * N) +
            2.0 * U * J[i] * J[j] / (N * N * N);
}

/* P-wave angular density, Eq. 4, term by term in the paper's order.
 * Its integral over [-1,1]^2 x [-pi,pi] is 1 for every parameter value. */
static void leaf_pwave(const orc_model* m, const orc_node* nd, const double* xe,
                       const double* th, int order, val_t* o) {
  int np = m->npar;
  double ctl = xe[nd->dim[0]], ctk = xe[nd->dim[1]], phi = xe[nd->dim[2]];
  double FL = th[nd->par[0]], S3 = th[nd->par[1]], S4 = th[nd->par[2]],
         S5 = th[nd->par[3]], AFB = th[nd->par[4]], S7 = th[nd->par[5]],
         S8 = th[nd->par[6]], S9 = th[nd->par[7]];
  double c = 9.0 / (32.0 * M_PI);
  double sin2tl = 1.0 - ctl * ctl; /* sin^2 theta_l */
  double sin2tk = 1.0 - ctk * ctk; /* sin^2 theta_K */
  double stl = sqrt(sin2tl), stk = sqrt(sin2tk);
  double cos2tl = 2.0 * ctl * ctl - 1.0;
  double sin2thl = 2.0 * stl * ctl; /* sin 2 theta_l */
  double sin2thk = 2.0 * stk * ctk; /* sin 2 theta_K */
  double cphi = cos(phi), sphi = sin(phi), c2phi = cos(2.0 * phi),
         s2phi = sin(2.0 * phi);
  /* the eleven angular terms f_i of Eq. 4 */
  double f1 = 0.75 * sin2tk;
  double f2 = ctk * ctk;
  double f3 = 0.25 * sin2tk * cos2tl;
  double f4 = ctk * ctk * cos2tl;
  double f5 = sin2tk * sin2tl * c2phi;
  double f6 = sin2thk * sin2thl * cphi;
  double f7 = sin2thk * stl * cphi;
  double f8 = 4.0 / 3.0 * sin2tk * ctl;
  double f9 = sin2thk * stl * sphi;
  double f10 = sin2thk * sin2thl * sphi;
  double f11 = sin2tk * sin2tl * s2phi;
  o->v = c * ((1.0 - FL) * f1 + FL * f2 + (1.0 - FL) * f3 - FL * f4 + S3 * f5 +
              S4 * f6 + S5 * f7 + AFB * f8 + S7 * f9 + S8 * f10 + S9 * f11);
  if (order >= 1) {
    o->g[nd->par[0]] += c * (-f1 + f2 - f3 - f4);
    o->g[nd->par[1]] += c * f5;
    o->g[nd->par[2]] += c * f6;
    o->g[nd->par[3]] += c * f7;
    o->g[nd->par[4]] += c * f8;
    o->g[nd->par[5]] += c * f9;
    o->g[nd->par[6]] += c * f10;
    o->g[nd->par[7]] += c * f11;
  }
  (void)np; /* linear in its parameters: second derivatives vanish */
}

/* ------------------------------------------------------------------ */
/* tree                                                                */
/* ------------------------------------------------------------------ */

static void eval_node(const orc_model* m, int id, const double* xe,
                      const double* th, int order, val_t* o) {
  const orc_node* nd = &m->node[id];
  int np = m->npar;
  clear_val(o, order, np);
  switch (nd->kind) {
    case ORC_GAUSS:
      leaf_gauss(m, nd, xe, th, order, o);
      return;
    case ORC_EXP:
      leaf_exp(m, nd, xe, th, order, o);
      return;
    case ORC_CHEB:
      leaf_cheb(m, nd, xe, th, order, o);
      return;
    case ORC_PWAVE:
      leaf_pwave(m, nd, xe, th, order, o);
      return;
    case ORC_PROD: {
      /* (AB)' = A'B + AB';  (AB)'' = A''B + AB'' + A'B'^T + B'A'^T */
      val_t* c = (val_t*)malloc(sizeof(val_t));
      eval_node(m, nd->child[0], xe, th, order, o);
      for (int k = 1; k < nd->nchild; ++k) {
        eval_node(m, nd->child[k], xe, th, order, c);
        if (order >= 2)
          for (int a = 0; a < np; ++a)
            for (int b = 0; b < np; ++b)
              o->h[a * np + b] = o->h[a * np + b] * c->v + o->v * c->h[a * np + b] +
                                 o->g[a] * c->g[b] + c->g[a] * o->g[b];
        if (order >= 1)
          for (int a = 0; a < np; ++a) o->g[a] = o->g[a] * c->v + o->v * c->g[a];
        o->v *= c->v;
      }
      free(c);
      return;
    }
    case ORC_SUM: {
      /* P = f A + (1 - f) B, a density only for 0 <= f <= 1 */
      val_t* A = (val_t*)malloc(sizeof(val_t));
      val_t* B = (val_t*)malloc(sizeof(val_t));
      int pf = nd->par[0];
      double f = th[pf];
      if (!(f >= 0.0 && f <= 1.0)) { /* not a mixture of densities */
        o->v = NAN;
        free(A);
        free(B);
        return;
      }
      eval_node(m, nd->child[0], xe, th, order, A);
      eval_node(m, nd->child[1], xe, th, order, B);
      o->v = f * A->v + (1.0 - f) * B->v;
      if (order >= 1) {
        for (int a = 0; a < np; ++a) o->g[a] = f * A->g[a] + (1.0 - f) * B->g[a];
        o->g[pf] += A->v - B->v;
      }
      if (order >= 2) {
        for (int a = 0; a < np; ++a)
          for (int b = 0; b < np; ++b)
            o->h[a * np + b] = f * A->h[a * np + b] + (1.0 - f) * B->h[a * np + b];
        for (int a = 0; a < np; ++a) {
          o->h[pf * np + a] += A->g[a] - B->g[a];
          o->h[a * np + pf] += A->g[a] - B->g[a];
        }
      }
      free(A);
      free(B);
      return;
    }
    default:
      o->v = NAN;
      return;
  }
}

void orc_pdf(const orc_model* m, long n, const double* x, const double* theta,
             double* out) {
  val_t* o = (val_t*)malloc(sizeof(val_t));
  double xe[ORC_MAXD];
  for (long i = 0; i < n; ++i) {
    for (int d = 0; d < m->ndim; ++d) xe[d] = x[(long)d * n + i];
    eval_node(m, m->root, xe, theta, 0, o);
    out[i] = o->v;
  }
  free(o);
}

/* ------------------------------------------------------------------ */
/* NLL, gradient, Hessian                                              */
/* ------------------------------------------------------------------ */

/* Neumaier's improvement of Kahan summation: running sum s, compensation c. */
static void nadd(double* s, double* c, double x) {
  double t = *s + x;
  if (fabs(*s) >= fabs(x))
    *c += (*s - t) + x;
  else
    *c += (x - t) + *s;
  *s = t;
}

long orc_nll(const orc_model* m, long n, const double* x, const double* w,
             const double* theta, int order, double* nll, double* grad,
             double* hess) {
  int np = m->npar;
  double s0 = 0.0, c0 = 0.0;
  double* gs = (double*)calloc(2 * NP, sizeof(double));
  double* hs = (double*)calloc(2 * NP * NP, sizeof(double));
  val_t* o = (val_t*)malloc(sizeof(val_t));
  double xe[ORC_MAXD], sc[NP];
  long bad = 0;
  for (long i = 0; i < n; ++i) {
    for (int d = 0; d < m->ndim; ++d) xe[d] = x[(long)d * n + i];
    double wi = w ? w[i] : 1.0;
    eval_node(m, m->root, xe, theta, order, o);
    double v = o->v;
    if (!(v > 0.0) || !isfinite(v)) {
      ++bad;
      continue;
    }
    nadd(&s0, &c0, -wi * log(v));
    if (order >= 1)
      for (int a = 0; a < np; ++a) {
        sc[a] = o->g[a] / v; /* d ln P / d theta_a */
        nadd(&gs[a], &gs[NP + a], -wi * sc[a]);
      }
    if (order >= 2)
      for (int a = 0; a < np; ++a)
        for (int b = 0; b < np; ++b)
          nadd(&hs[a * np + b], &hs[NP * NP + a * np + b],
               wi * (sc[a] * sc[b] - o->h[a * np + b] / v));
  }
  *nll = bad ? INFINITY : s0 + c0;
  if (order >= 1 && grad)
    for (int a = 0; a < np; ++a) grad[a] = bad ? 0.0 : gs[a] + gs[NP + a];
  if (order >= 2 && hess)
    for (int a = 0; a < np * np; ++a) hess[a] = bad ? 0.0 : hs[a] + hs[NP * NP + a];
  free(o);
  free(gs);
  free(hs);
  return bad;
}

/* Sum over events of w_i^2 s_i s_i^T with s_i = d ln P(x_i) / d theta
   (all parameters): the variance of the weighted score, the middle factor
   of the weighted-fit covariance H^-1 W2 H^-1.  Neumaier sums; any P <= 0
   gives W2 = 0 and is counted in the return value. */
long orc_w2(const orc_model* m, long n, const double* x, const double* w,
            const double* theta, double* w2) {
  int np = m->npar;
  double* ss = (double*)calloc(2 * NP * NP, sizeof(double));
  val_t* o = (val_t*)malloc(sizeof(val_t));
  double xe[ORC_MAXD], sc[NP];
  long bad = 0;
  for (long i = 0; i < n; ++i) {
    for (int d = 0; d < m->ndim; ++d) xe[d] = x[(long)d * n + i];
    double wi = w ? w[i] : 1.0;
    eval_node(m, m->root, xe, theta, 1, o);
    double v = o->v;
    if (!(v > 0.0) || !isfinite(v)) {
      ++bad;
      continue;
    }
    for (int a = 0; a < np; ++a) sc[a] = o->g[a] / v;
    for (int a = 0; a < np; ++a)
      for (int b = 0; b < np; ++b)
        nadd(&ss[a * np + b], &ss[NP * NP + a * np + b], wi * wi * sc[a] * sc[b]);
  }
  for (int a = 0; a < np * np; ++a) w2[a] = bad ? 0.0 : ss[a] + ss[NP * NP + a];
  free(o);
  free(ss);
  return bad;
}

/* ------------------------------------------------------------------ */
/* pseudo-experiment generation                                        */
/* ------------------------------------------------------------------ */

/* Philox4x64 with 10 rounds (Salmon, Moraes, Dror and Shaw, "Parallel
   random numbers: as easy as 1, 2, 3", SC11): a counter-based generator.
   Each round multiplies words 0 and 2 by fixed odd constants, keeps the
   128-bit products' halves and mixes them with words 1 and 3 and the key;
   the key is advanced by two Weyl constants between rounds. */
void orc_philox4x64(const unsigned long long ctr[4], const unsigned long long key[2],
                    unsigned long long out[4]) {
  const unsigned long long M0 = 0xD2E7470EE14C6C93ULL, M1 = 0xCA5A826395121157ULL;
  const unsigned long long W0 = 0x9E3779B97F4A7C15ULL, W1 = 0xBB67AE8584CAA73BULL;
  unsigned long long x0 = ctr[0], x1 = ctr[1], x2 = ctr[2], x3 = ctr[3];
  unsigned long long k0 = key[0], k1 = key[1];
  for (int r = 0; r < 10; ++r) {
    unsigned __int128 p0 = (unsigned __int128)M0 * x0;
    unsigned __int128 p1 = (unsigned __int128)M1 * x2;
    unsigned long long hi0 = (unsigned long long)(p0 >> 64), lo0 = (unsigned long long)p0;
    unsigned long long hi1 = (unsigned long long)(p1 >> 64), lo1 = (unsigned long long)p1;
    x0 = hi1 ^ x1 ^ k0;
    x1 = lo1;
    x2 = hi0 ^ x3 ^ k1;
    x3 = lo0;
    k0 += W0;
    k1 += W1;
  }
  out[0] = x0;
  out[1] = x1;
  out[2] = x2;
  out[3] = x3;
}

/* The uniform stream of one event: blocks b = 0, 1, .. of Philox with
   counter (b, event, 0, 0) and key (seed, 0), four 64-bit words each, each
   word giving u = (top 53 bits + 1/2) / 2^53 in (0, 1). */
typedef struct {
  unsigned long long key[2], ctr[4], buf[4];
  int pos;
} ustream;

static void us_init(ustream* s, unsigned long long seed, long event) {
  s->key[0] = seed;
  s->key[1] = 0;
  s->ctr[0] = 0;
  s->ctr[1] = (unsigned long long)event;
  s->ctr[2] = s->ctr[3] = 0;
  s->pos = 4;
}

static double us_next(ustream* s) {
  if (s->pos == 4) {
    orc_philox4x64(s->ctr, s->key, s->buf);
    s->ctr[0] += 1;
    s->pos = 0;
  }
  unsigned long long r = s->buf[s->pos++];
  return ((double)(r >> 11) + 0.5) * (1.0 / 9007199254740992.0);
}

#define ORC_GEN_CAP 65536 /* accept-reject attempts per draw */

/* Draws the dimensions of node id into xe; returns 0, or 1 if a draw hit
   the attempt cap.  Sums pick a child with probability f / 1 - f; products
   draw every child; leaves draw their dimensions: the Gaussian by the
   Box-Muller transform with rejection outside the range, the exponential by
   its inverse distribution function, the Chebyshev series and the P-wave
   density by accept-reject under the sum of the absolute values of their
   terms' coefficients times the terms' maxima. */
static int gen_node(const orc_model* m, int id, const double* th, ustream* s, double* xe) {
  const orc_node* nd = &m->node[id];
  switch (nd->kind) {
    case ORC_SUM: {
      double f = th[nd->par[0]];
      double u = us_next(s);
      return gen_node(m, nd->child[u < f ? 0 : 1], th, s, xe);
    }
    case ORC_PROD: {
      int bad = 0;
      for (int c = 0; c < nd->nchild; ++c) bad |= gen_node(m, nd->child[c], th, s, xe);
      return bad;
    }
    case ORC_GAUSS: {
      int d = nd->dim[0];
      double lo = m->lo[d], hi = m->hi[d], mu = th[nd->par[0]], sg = th[nd->par[1]];
      for (int a = 0; a < ORC_GEN_CAP; ++a) {
        double u1 = us_next(s), u2 = us_next(s);
        double x = mu + sg * (sqrt(-2.0 * log(u1)) * cos(2.0 * M_PI * u2));
        if (x >= lo && x <= hi) {
          xe[d] = x;
          return 0;
        }
      }
      xe[d] = lo;
      return 1;
    }
    case ORC_EXP: {
      int d = nd->dim[0];
      double lo = m->lo[d], hi = m->hi[d], lam = th[nd->par[0]], L = hi - lo;
      double u = us_next(s);
      double x = lam == 0.0 ? lo + u * L : lo + log1p(u * expm1(lam * L)) / lam;
      xe[d] = x < lo ? lo : (x > hi ? hi : x);
      return 0;
    }
    case ORC_CHEB: {
      int d = nd->dim[0], k = nd->npar;
      double lo = m->lo[d], hi = m->hi[d], L = hi - lo, env = 1.0;
      for (int j = 0; j < k; ++j) env += fabs(th[nd->par[j]]);
      for (int a = 0; a < ORC_GEN_CAP; ++a) {
        double u1 = us_next(s), u2 = us_next(s);
        double x = lo + u1 * L;
        double t = (2.0 * x - lo - hi) / L, tm = 1.0, tj = t, v = 1.0;
        for (int j = 1; j <= k; ++j) {
          v += th[nd->par[j - 1]] * tj;
          double tn = 2.0 * t * tj - tm;
          tm = tj;
          tj = tn;
        }
        if (u2 * env <= v) {
          xe[d] = x;
          return 0;
        }
      }
      xe[d] = lo;
      return 1;
    }
    case ORC_PWAVE: {
      double FL = th[nd->par[0]];
      double env = 0.75 * fabs(1.0 - FL) + fabs(FL) + 0.25 * fabs(1.0 - FL) + fabs(FL) +
                   4.0 / 3.0 * fabs(th[nd->par[4]]);
      for (int k = 1; k < 8; ++k)
        if (k != 4) env += fabs(th[nd->par[k]]);
      env *= 9.0 / (32.0 * M_PI); /* the value below carries the same factor */
      val_t* o = (val_t*)malloc(sizeof(val_t));
      int bad = 1;
      for (int a = 0; a < ORC_GEN_CAP; ++a) {
        double u1 = us_next(s), u2 = us_next(s), u3 = us_next(s), u4 = us_next(s);
        xe[nd->dim[0]] = 2.0 * u1 - 1.0;
        xe[nd->dim[1]] = 2.0 * u2 - 1.0;
        xe[nd->dim[2]] = M_PI * (2.0 * u3 - 1.0);
        leaf_pwave(m, nd, xe, th, 0, o);
        if (u4 * env <= o->v) {
          bad = 0;
          break;
        }
      }
      free(o);
      if (bad) {
        xe[nd->dim[0]] = m->lo[nd->dim[0]];
        xe[nd->dim[1]] = m->lo[nd->dim[1]];
        xe[nd->dim[2]] = m->lo[nd->dim[2]];
      }
      return bad;
    }
  }
  return 1;
}

long orc_generate(const orc_model* m, long i0, long n, unsigned long long seed,
                  const double* theta, double* x) {
  long bad = 0;
  double xe[ORC_MAXD];
  for (long i = 0; i < n; ++i) {
    ustream s;
    us_init(&s, seed, i0 + i);
    for (int d = 0; d < m->ndim; ++d) xe[d] = m->lo[d];
    bad += gen_node(m, m->root, theta, &s, xe);
    for (int d = 0; d < m->ndim; ++d) x[(long)d * n + i] = xe[d];
  }
  return bad;
}

/* ------------------------------------------------------------------ */
/* BFGS fit                                                            */
/* ------------------------------------------------------------------ */

/* Inverse of a symmetric positive-definite matrix by Cholesky. */
static int chol_inv(int n, const double* A, double* Ai) {
  double L[NP * NP];
  memset(L, 0, sizeof(L));
  for (int j = 0; j < n; ++j) {
    double s = A[j * n + j];
    for (int k = 0; k < j; ++k) s -= L[j * n + k] * L[j * n + k];
    if (!(s > 0.0)) return -1;
    L[j * n + j] = sqrt(s);
    for (int i = j + 1; i < n; ++i) {
      double t = A[i * n + j];
      for (int k = 0; k < j; ++k) t -= L[i * n + k] * L[j * n + k];
      L[i * n + j] = t / L[j * n + j];
    }
  }
  /* A^{-1} column by column: solve L y = e_c, then L^T x = y */
  for (int c = 0; c < n; ++c) {
    double y[NP];
    for (int i = 0; i < n; ++i) {
      double t = (i == c) ? 1.0 : 0.0;
      for (int k = 0; k < i; ++k) t -= L[i * n + k] * y[k];
      y[i] = t / L[i * n + i];
    }
    for (int i = n - 1; i >= 0; --i) {
      double t = y[i];
      for (int k = i + 1; k < n; ++k) t -= L[k * n + i] * Ai[k * n + c];
      Ai[i * n + c] = t / L[i * n + i];
    }
  }
  return 0;
}

typedef struct {
  const orc_model* m;
  long n;
  const double* x;
  const double* w;
  int nf;
  int idx[NP];
  double th[NP]; /* full parameter vector; free entries overwritten */
  int n_eval;
} fit_ctx;

static double fc_eval(fit_ctx* fc, const double* xf, int order, double* gf,
                      double* Hf) {
  double g[NP], H[NP * NP], nll;
  int np = fc->m->npar;
  for (int k = 0; k < fc->nf; ++k) fc->th[fc->idx[k]] = xf[k];
  orc_nll(fc->m, fc->n, fc->x, fc->w, fc->th, order, &nll, g, H);
  fc->n_eval++;
  if (order >= 1)
    for (int a = 0; a < fc->nf; ++a) gf[a] = g[fc->idx[a]];
  if (order >= 2)
    for (int a = 0; a < fc->nf; ++a)
      for (int b = 0; b < fc->nf; ++b)
        Hf[a * fc->nf + b] = H[fc->idx[a] * np + fc->idx[b]];
  return nll;
}

static double quad_form(int n, const double* V, const double* g) {
  double s = 0.0;
  for (int a = 0; a < n; ++a)
    for (int b = 0; b < n; ++b) s += g[a] * V[a * n + b] * g[b];
  return s;
}

int orc_fit(const orc_model* m, long n, const double* x, const double* w,
            double* theta, const int* free_mask, const orc_fit_opts* opts,
            double* cov, orc_fit_info* info) {
  fit_ctx fc;
  memset(&fc, 0, sizeof(fc));
  fc.m = m;
  fc.n = n;
  fc.x = x;
  fc.w = w;
  for (int k = 0; k < m->npar; ++k) {
    fc.th[k] = theta[k];
    if (free_mask[k]) fc.idx[fc.nf++] = k;
  }
  int nf = fc.nf;
  double xf[NP], g[NP], H[NP * NP], V[NP * NP], p[NP], xt[NP], gt[NP];
  for (int k = 0; k < nf; ++k) xf[k] = theta[fc.idx[k]];
  memset(info, 0, sizeof(*info));

  double f = fc_eval(&fc, xf, 2, g, H);
  if (!isfinite(f)) {
    info->status = 2;
    info->nll = f;
    return -1;
  }
  /* initial metric: inverse of the analytic Hessian at the start */
  if (chol_inv(nf, H, V) != 0) {
    memset(V, 0, sizeof(V));
    for (int a = 0; a < nf; ++a)
      V[a * nf + a] = 1.0 / fmax(fabs(H[a * nf + a]), 1e-300);
  }
  int status = 1, it = 0;
  double edm = 0.5 * quad_form(nf, V, g);
  for (it = 0; it < opts->max_iter; ++it) {
    edm = 0.5 * quad_form(nf, V, g);
    if (edm < opts->edm_tol) {
      status = 0;
      break;
    }
    double gp = 0.0;
    for (int a = 0; a < nf; ++a) {
      p[a] = 0.0;
      for (int b = 0; b < nf; ++b) p[a] -= V[a * nf + b] * g[b];
      gp += g[a] * p[a];
    }
    if (!(gp < 0.0)) { /* metric lost positivity: restart from the Hessian */
      fc_eval(&fc, xf, 2, g, H);
      if (chol_inv(nf, H, V) != 0) {
        status = 3;
        break;
      }
      continue;
    }
    /* backtracking line search with the Armijo condition */
    double alpha = 1.0, ft = INFINITY;
    int ok = 0;
    for (int ls = 0; ls < 60; ++ls) {
      for (int a = 0; a < nf; ++a) xt[a] = xf[a] + alpha * p[a];
      ft = fc_eval(&fc, xt, 1, gt, NULL);
      if (isfinite(ft) && ft <= f + 1e-4 * alpha * gp + 1e-15 * fabs(f)) {
        ok = 1;
        break;
      }
      if (!isfinite(ft)) {
        alpha *= 0.25;
      } else {
        double aq = -gp * alpha * alpha / (2.0 * (ft - f - gp * alpha));
        alpha = fmin(fmax(aq, 0.1 * alpha), 0.5 * alpha);
      }
    }
    if (!ok) {
      status = (edm < 100.0 * opts->edm_tol) ? 0 : 2;
      break;
    }
    double s[NP], y[NP], Vy[NP], sy = 0.0, yVy = 0.0;
    for (int a = 0; a < nf; ++a) {
      s[a] = xt[a] - xf[a];
      y[a] = gt[a] - g[a];
      sy += s[a] * y[a];
    }
    for (int a = 0; a < nf; ++a) {
      Vy[a] = 0.0;
      for (int b = 0; b < nf; ++b) Vy[a] += V[a * nf + b] * y[b];
      yVy += y[a] * Vy[a];
    }
    if (sy > 0.0) { /* inverse-Hessian BFGS update */
      double c1 = (sy + yVy) / (sy * sy);
      for (int a = 0; a < nf; ++a)
        for (int b = 0; b < nf; ++b)
          V[a * nf + b] += c1 * s[a] * s[b] - (Vy[a] * s[b] + s[a] * Vy[b]) / sy;
    }
    for (int a = 0; a < nf; ++a) {
      xf[a] = xt[a];
      g[a] = gt[a];
    }
    f = ft;
  }
  info->n_iter = it;
  /* optional Newton polish with the analytic Hessian */
  for (int k = 0; k < opts->polish; ++k) {
    double Hi[NP * NP];
    fc_eval(&fc, xf, 2, g, H);
    if (chol_inv(nf, H, Hi) != 0) break;
    for (int a = 0; a < nf; ++a) {
      xt[a] = xf[a];
      for (int b = 0; b < nf; ++b) xt[a] -= Hi[a * nf + b] * g[b];
    }
    double fn = fc_eval(&fc, xt, 1, gt, NULL);
    if (!isfinite(fn)) break;
    for (int a = 0; a < nf; ++a) xf[a] = xt[a];
    f = fn;
  }
  /* covariance: inverse Hessian of the NLL at the minimum */
  f = fc_eval(&fc, xf, 2, g, H);
  if (chol_inv(nf, H, cov) != 0) status = 3;
  else edm = 0.5 * quad_form(nf, cov, g);
  for (int k = 0; k < nf; ++k) theta[fc.idx[k]] = xf[k];
  info->nll = f;
  info->edm = edm;
  info->n_eval = fc.n_eval;
  info->status = status;
  return 0;
}
