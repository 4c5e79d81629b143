// Model description -> plan: validation, expansion of the tree into a mixture
// of products, canonical ordering and the constant/moment layout.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "hess.h"
#include "host.h"

namespace uml {

namespace {

struct Term {
  std::vector<std::pair<int, int>> frac;  // (parameter, +1 for f / -1 for 1 - f)
  std::vector<int> leaves;                // node indices
};

int expected_params(int kind) {
  switch (kind) {
    case UML_GAUSS: return 2;
    case UML_EXP: return 1;
    case UML_PWAVE: return 8;
    case UML_SUM: return 1;
    case UML_PROD: return 0;
    default: return -1;
  }
}

int n_leaf_dims(int kind) { return kind == UML_PWAVE ? 3 : (kind == UML_PROD || kind == UML_SUM) ? 0 : 1; }

bool expand(const uml_model_desc* d, int id, int depth, std::vector<Term>& out, std::string& err) {
  if (depth > UML_MAX_NODES) {
    err = "model tree has a cycle or is too deep";
    return false;
  }
  const uml_node& nd = d->nodes[id];
  if (nd.kind == UML_SUM) {
    std::vector<Term> a, b;
    if (!expand(d, nd.children[0], depth + 1, a, err) || !expand(d, nd.children[1], depth + 1, b, err))
      return false;
    for (auto& t : a) {
      t.frac.insert(t.frac.begin(), {nd.params[0], +1});
      out.push_back(t);
    }
    for (auto& t : b) {
      t.frac.insert(t.frac.begin(), {nd.params[0], -1});
      out.push_back(t);
    }
    return true;
  }
  if (nd.kind == UML_PROD) {
    std::vector<Term> acc(1);
    for (int k = 0; k < nd.n_children; ++k) {
      std::vector<Term> ch, nxt;
      if (!expand(d, nd.children[k], depth + 1, ch, err)) return false;
      for (const auto& x : acc)
        for (const auto& y : ch) {
          Term t = x;
          t.frac.insert(t.frac.end(), y.frac.begin(), y.frac.end());
          t.leaves.insert(t.leaves.end(), y.leaves.begin(), y.leaves.end());
          nxt.push_back(t);
        }
      acc.swap(nxt);
    }
    out.insert(out.end(), acc.begin(), acc.end());
    return true;
  }
  Term t;
  t.leaves.push_back(id);
  out.push_back(t);
  return true;
}

int leaf_kind(int uml_kind) {
  switch (uml_kind) {
    case UML_GAUSS: return FK_GAUSS;
    case UML_EXP: return FK_EXP;
    case UML_CHEB: return FK_CHEB;
    default: return FK_PWAVE;
  }
}

char kind_letter(int fk) { return fk == FK_GAUSS ? 'G' : fk == FK_EXP ? 'E' : fk == FK_CHEB ? 'C' : 'P'; }

}  // namespace

std::string plan_signature(const Plan& P) {
  std::string s;
  for (int c = 0; c < P.ncomp; ++c) {
    if (c) s += "|";
    for (int j = 0; j < P.comp[c].nfac; ++j) {
      const FactorPlan& F = P.fac[P.comp[c].fac[j]];
      if (F.kind == FK_PWAVE && F.pre >= 0) {  // terms read from columns pre .. pre + 8
        s += "Q" + std::to_string(F.pre);
      } else if (F.kind == FK_PWAVE) {
        s += kind_letter(F.kind);
        for (int k = 0; k < 3; ++k) s += std::to_string(F.dim[k]);
      } else {
        s += kind_letter(F.kind);
        s += std::to_string(F.dim[0]);
        if (F.kind == FK_CHEB) s += "." + std::to_string(F.order);
      }
    }
  }
  return s;
}

int build_plan(const uml_model_desc* d, Plan& P, std::string& err) {
  std::memset(&P, 0, sizeof(P));
  if (!d) {
    err = "null model description";
    return UML_E_INVALID;
  }
  if (d->n_dims < 1 || d->n_dims > UML_MAX_DIMS || !d->dims) {
    err = "n_dims must be in 1.." + std::to_string(UML_MAX_DIMS);
    return UML_E_INVALID;
  }
  if (d->n_params < 0 || d->n_params > UML_MAX_PARAMS || (d->n_params && !d->params)) {
    err = "n_params must be in 0.." + std::to_string(UML_MAX_PARAMS);
    return UML_E_INVALID;
  }
  if (d->n_nodes < 1 || d->n_nodes > UML_MAX_NODES || !d->nodes || d->root < 0 ||
      d->root >= d->n_nodes) {
    err = "bad node list or root";
    return UML_E_INVALID;
  }
  if (d->precision != UML_FP64 && d->precision != UML_MIXED) {
    err = "precision must be UML_FP64 or UML_MIXED";
    return UML_E_INVALID;
  }
  for (int k = 0; k < d->n_dims; ++k)
    if (!(d->dims[k].hi > d->dims[k].lo) || !std::isfinite(d->dims[k].lo) ||
        !std::isfinite(d->dims[k].hi)) {
      err = "dimension " + std::to_string(k) + ": need finite lo < hi";
      return UML_E_INVALID;
    }
  for (int k = 0; k < d->n_params; ++k)
    if (!std::isfinite(d->params[k].value)) {
      err = "parameter " + std::to_string(k) + " has a non-finite value";
      return UML_E_INVALID;
    }
  // node checks
  for (int i = 0; i < d->n_nodes; ++i) {
    const uml_node& nd = d->nodes[i];
    const std::string where = "node " + std::to_string(i) + ": ";
    if (nd.kind < UML_GAUSS || nd.kind > UML_SUM) {
      err = where + "unknown kind";
      return UML_E_INVALID;
    }
    int np = expected_params(nd.kind);
    if (nd.kind == UML_CHEB) {
      if (nd.n_params < 1 || nd.n_params > kMaxCheb) {
        err = where + "a Chebyshev series takes 1.." + std::to_string(kMaxCheb) + " coefficients";
        return UML_E_INVALID;
      }
    } else if (nd.n_params != np) {
      err = where + "expected " + std::to_string(np) + " parameters";
      return UML_E_INVALID;
    }
    for (int k = 0; k < nd.n_params; ++k)
      if (nd.params[k] < 0 || nd.params[k] >= d->n_params) {
        err = where + "parameter index out of range";
        return UML_E_INVALID;
      }
    for (int k = 0; k < n_leaf_dims(nd.kind); ++k)
      if (nd.dims[k] < 0 || nd.dims[k] >= d->n_dims) {
        err = where + "dimension index out of range";
        return UML_E_INVALID;
      }
    if (nd.kind == UML_SUM && nd.n_children != 2) {
      err = where + "a sum has exactly two children";
      return UML_E_INVALID;
    }
    if (nd.kind == UML_PROD && (nd.n_children < 2 || nd.n_children > 4)) {
      err = where + "a product has 2..4 children";
      return UML_E_INVALID;
    }
    if (nd.kind == UML_SUM || nd.kind == UML_PROD)
      for (int k = 0; k < nd.n_children; ++k)
        if (nd.children[k] < 0 || nd.children[k] >= d->n_nodes || nd.children[k] == i) {
          err = where + "child index out of range";
          return UML_E_INVALID;
        }
    if (nd.kind == UML_PWAVE) {
      const double want_lo[3] = {-1.0, -1.0, -M_PI}, want_hi[3] = {1.0, 1.0, M_PI};
      for (int k = 0; k < 3; ++k) {
        const uml_dim& dm = d->dims[nd.dims[k]];
        if (std::fabs(dm.lo - want_lo[k]) > 1e-12 || std::fabs(dm.hi - want_hi[k]) > 1e-12) {
          err = where + "the P-wave density needs ranges [-1,1], [-1,1], [-pi,pi]";
          return UML_E_INVALID;
        }
      }
      if (nd.dims[0] == nd.dims[1] || nd.dims[0] == nd.dims[2] || nd.dims[1] == nd.dims[2]) {
        err = where + "the P-wave density needs three distinct dimensions";
        return UML_E_INVALID;
      }
    }
  }
  std::vector<Term> terms;
  if (!expand(d, d->root, 0, terms, err)) return UML_E_INVALID;
  if ((int)terms.size() > kMaxComp) {
    err = "the model expands into " + std::to_string(terms.size()) + " components (max " +
          std::to_string(kMaxComp) + ")";
    return UML_E_UNSUPPORTED;
  }
  // every component covers each dimension exactly once
  for (size_t c = 0; c < terms.size(); ++c) {
    std::vector<int> seen(d->n_dims, 0);
    if ((int)terms[c].leaves.size() > kMaxFacPerComp) {
      err = "a component has more than " + std::to_string(kMaxFacPerComp) + " factors";
      return UML_E_UNSUPPORTED;
    }
    for (int id : terms[c].leaves) {
      const uml_node& nd = d->nodes[id];
      for (int k = 0; k < n_leaf_dims(nd.kind); ++k) seen[nd.dims[k]]++;
    }
    for (int k = 0; k < d->n_dims; ++k)
      if (seen[k] != 1) {
        err = "component " + std::to_string(c) + " uses dimension " + std::to_string(k) + " " +
              std::to_string(seen[k]) + " times (products must cover every dimension once)";
        return UML_E_INVALID;
      }
  }
  // canonical dimension numbering: Gaussian/exponential dimensions first,
  // then P-wave dimensions in the P-wave's order, then the rest
  std::vector<int> kdim(d->n_dims, -1);
  int next = 0;
  auto number = [&](int ud) {
    if (kdim[ud] < 0) kdim[ud] = next++;
  };
  for (const auto& t : terms)
    for (int id : t.leaves)
      if (d->nodes[id].kind == UML_GAUSS || d->nodes[id].kind == UML_EXP) number(d->nodes[id].dims[0]);
  for (const auto& t : terms)
    for (int id : t.leaves)
      if (d->nodes[id].kind == UML_PWAVE)
        for (int k = 0; k < 3; ++k) number(d->nodes[id].dims[k]);
  for (const auto& t : terms)
    for (int id : t.leaves)
      if (d->nodes[id].kind == UML_CHEB) number(d->nodes[id].dims[0]);
  for (int k = 0; k < d->n_dims; ++k) number(k);
  // factors inside a component by (kind, first kernel dimension); components
  // by their kind string
  auto fkey = [&](int id) {
    const uml_node& nd = d->nodes[id];
    return std::make_pair(leaf_kind(nd.kind), kdim[nd.dims[0]]);
  };
  for (auto& t : terms)
    std::stable_sort(t.leaves.begin(), t.leaves.end(), [&](int a, int b) { return fkey(a) < fkey(b); });
  auto kstr = [&](const Term& t) {
    std::string s;
    for (int id : t.leaves) s += kind_letter(leaf_kind(d->nodes[id].kind));
    return s;
  };
  std::stable_sort(terms.begin(), terms.end(), [&](const Term& a, const Term& b) { return kstr(a) < kstr(b); });

  // shifts: dimensions carrying a Gaussian or an exponential are evaluated as
  // x' = x - xref with xref an FP32 value near the data (the first Gaussian's
  // mean, else the range midpoint), so that x' is exact in FP32 and the
  // exponents stay small.
  P.ndim = d->n_dims;
  for (int ud = 0; ud < d->n_dims; ++ud) {
    P.dim_of_user[ud] = kdim[ud];
    P.user_of_dim[kdim[ud]] = ud;
    P.lo[kdim[ud]] = d->dims[ud].lo;
    P.hi[kdim[ud]] = d->dims[ud].hi;
  }
  std::vector<int> shifted(P.ndim, 0), pwave_dim(P.ndim, 0);
  std::vector<double> gmean(P.ndim, NAN);
  for (const auto& t : terms)
    for (int id : t.leaves) {
      const uml_node& nd = d->nodes[id];
      if (nd.kind == UML_GAUSS || nd.kind == UML_EXP) shifted[kdim[nd.dims[0]]] = 1;
      if (nd.kind == UML_GAUSS && std::isnan(gmean[kdim[nd.dims[0]]]))
        gmean[kdim[nd.dims[0]]] = d->params[nd.params[0]].value;
      if (nd.kind == UML_PWAVE)
        for (int k = 0; k < 3; ++k) pwave_dim[kdim[nd.dims[k]]] = 1;
    }
  for (int kd = 0; kd < P.ndim; ++kd) {
    if (shifted[kd] && pwave_dim[kd]) {
      err = "a dimension of the P-wave density cannot also carry a Gaussian or exponential";
      return UML_E_UNSUPPORTED;
    }
    double ref = 0.0;
    if (shifted[kd]) {
      ref = std::isnan(gmean[kd]) ? 0.5 * (P.lo[kd] + P.hi[kd]) : gmean[kd];
      ref = std::min(std::max(ref, P.lo[kd]), P.hi[kd]);
      ref = double(float(ref));
    }
    P.xref[kd] = ref;
  }

  // layout
  struct T3 {
    int par, mom, ec;
  };
  std::vector<T3> gterms;
  P.ncomp = (int)terms.size();
  int cst = 0, ecst = 0, mom = 1;
  for (int c = 0; c < P.ncomp; ++c) {
    CompPlan& C = P.comp[c];
    const Term& t = terms[c];
    if ((int)t.frac.size() > 8) {
      err = "too many nested sums";
      return UML_E_UNSUPPORTED;
    }
    C.nfrac = (int)t.frac.size();
    C.cst_lk2 = cst;
    cst += kCompCst;
    C.slot_r = mom++;
    for (int k = 0; k < C.nfrac; ++k) {
      C.frac_par[k] = t.frac[k].first;
      C.frac_sign[k] = t.frac[k].second;
      C.frac_ec[k] = ecst++;
      gterms.push_back({C.frac_par[k], C.slot_r, C.frac_ec[k]});
    }
    C.nfac = (int)t.leaves.size();
    for (int j = 0; j < C.nfac; ++j) {
      if (P.nfac >= kMaxFac) {
        err = "too many factors";
        return UML_E_UNSUPPORTED;
      }
      const uml_node& nd = d->nodes[t.leaves[j]];
      FactorPlan& F = P.fac[P.nfac];
      F.kind = leaf_kind(nd.kind);
      F.order = nd.kind == UML_CHEB ? nd.n_params : 0;
      for (int k = 0; k < n_leaf_dims(nd.kind); ++k) {
        F.dim[k] = kdim[nd.dims[k]];
        F.lo[k] = P.lo[F.dim[k]];
        F.hi[k] = P.hi[F.dim[k]];
      }
      for (int k = 0; k < nd.n_params; ++k) F.par[k] = nd.params[k];
      F.xref = P.xref[F.dim[0]];
      F.pre = -1;
      F.cst = cst;
      F.ecst = ecst;
      F.mom = mom;
      // gradient terms (see EpiTerm); R = the component's responsibility sum
      switch (F.kind) {
        case FK_GAUSS:  // mu: M_d, R; sigma: M_dd, R, M_d
          gterms.push_back({F.par[0], mom, ecst});
          gterms.push_back({F.par[0], C.slot_r, ecst + 1});
          gterms.push_back({F.par[1], mom + 1, ecst + 2});
          gterms.push_back({F.par[1], C.slot_r, ecst + 3});
          gterms.push_back({F.par[1], mom, ecst + 4});
          break;
        case FK_EXP:
          gterms.push_back({F.par[0], mom, ecst});
          gterms.push_back({F.par[0], C.slot_r, ecst + 1});
          break;
        case FK_CHEB:
          for (int k = 0; k < F.order; ++k) {
            gterms.push_back({F.par[k], mom + k, ecst + k});
            gterms.push_back({F.par[k], C.slot_r, ecst + F.order + k});
          }
          break;
        case FK_PWAVE:
          for (int k = 0; k < 8; ++k) gterms.push_back({F.par[k], mom + k, ecst + k});
          break;
      }
      cst += fk_ncst(F.kind, F.order);
      ecst += fk_necst(F.kind, F.order);
      mom += fk_nmom(F.kind, F.order);
      C.fac[j] = P.nfac++;
    }
  }
  if (cst > kMaxCst || ecst > kMaxECst || mom > kMaxK) {
    err = "model too large for the kernel constant layout";
    return UML_E_UNSUPPORTED;
  }
  P.ncst = cst;
  P.necst = ecst;
  P.K = mom;
  P.npar = d->n_params;
  if ((int)gterms.size() > kMaxTerms) {
    err = "model too large for the gradient term table";
    return UML_E_UNSUPPORTED;
  }
  std::stable_sort(gterms.begin(), gterms.end(), [](const T3& a, const T3& b) { return a.par < b.par; });
  P.nterm = (int)gterms.size();
  for (int k = 0; k < P.nterm; ++k) {
    P.term[k].mom = (short)gterms[k].mom;
    P.term[k].ec = (short)gterms[k].ec;
  }
  for (int p = 0, k = 0; p <= P.npar; ++p) {
    while (k < P.nterm && gterms[k].par < p) ++k;
    P.term_begin[p] = k;
  }
  P.nfree = 0;
  for (int k = 0; k < d->n_params; ++k) {
    P.free_pos[k] = -1;
    if (!d->params[k].fixed) {
      P.free_pos[k] = P.nfree;
      P.free_idx[P.nfree++] = k;
    }
  }
  P.precision = d->precision;
  // stored columns: the dimensions, then the precomputed P-wave terms
  P.ncol = P.ndim;
  P.pre_fac = -1;
  if (d->flags & ~UML_MODEL_PRECOMPUTE_ANGULAR) {
    err = "unknown model flags";
    return UML_E_INVALID;
  }
  if (d->flags & UML_MODEL_PRECOMPUTE_ANGULAR) {
    for (int f = 0; f < P.nfac; ++f) {
      if (P.fac[f].kind != FK_PWAVE) continue;
      if (P.pre_fac >= 0) {
        err = "precomputed angular terms need a model with one P-wave factor";
        return UML_E_UNSUPPORTED;
      }
      P.pre_fac = f;
      P.fac[f].pre = P.ncol;
      P.ncol += kPWaveTerms;
    }
    if (P.pre_fac < 0) {
      err = "precomputed angular terms need a P-wave factor";
      return UML_E_INVALID;
    }
    if (P.ncol > kMaxCols) {
      err = "too many stored columns";
      return UML_E_UNSUPPORTED;
    }
  }
  return UML_OK;
}

bool build_hess_plan(const Plan& P, HessPlan& H, std::string& err) {
  std::memset(&H, 0, sizeof(H));
  int nq = 0;
  for (int f = 0; f < P.nfac; ++f) {
    const FactorPlan& F = P.fac[f];
    H.q_off[f] = nq;
    nq += F.kind == FK_GAUSS ? 3 : F.kind == FK_EXP ? 1 : F.kind == FK_CHEB ? F.order * (F.order + 1) / 2 : 0;
  }
  H.nq = nq;
  // unit of every parameter in every component: fraction entry k -> 1000 + k,
  // factor j -> j (local index loc), absent -> -1
  std::vector<std::vector<int>> unit(P.ncomp, std::vector<int>(P.npar, -1)), loc = unit;
  for (int c = 0; c < P.ncomp; ++c) {
    const CompPlan& C = P.comp[c];
    for (int k = 0; k < C.nfrac; ++k) {
      if (unit[c][C.frac_par[k]] != -1) {
        err = "a parameter appears twice in one mixture component";
        return false;
      }
      unit[c][C.frac_par[k]] = 1000 + k;
    }
    for (int j = 0; j < C.nfac; ++j) {
      const FactorPlan& F = P.fac[C.fac[j]];
      const int np = F.kind == FK_GAUSS ? 2 : F.kind == FK_EXP ? 1 : F.kind == FK_CHEB ? F.order : 8;
      for (int m = 0; m < np; ++m) {
        if (unit[c][F.par[m]] != -1) {
          err = "a parameter appears twice in one mixture component";
          return false;
        }
        unit[c][F.par[m]] = j;
        loc[c][F.par[m]] = m;
      }
    }
  }
  int np = 0;
  for (int a = 0; a < P.nfree; ++a)
    for (int b = a; b < P.nfree; ++b, ++np) {
      H.pa[np] = short(a);
      H.pb[np] = short(b);
      const int pa = P.free_idx[a], pb = P.free_idx[b];
      for (int c = 0; c < kMaxComp; ++c) {
        signed char r = kRelAbsent;
        if (c < P.ncomp && unit[c][pa] >= 0 && unit[c][pb] >= 0) {
          const int ua = unit[c][pa], ub = unit[c][pb];
          if (ua != ub) {
            r = kRelProduct;
          } else if (ua >= 1000) {
            r = kRelZero;
          } else {
            const int fi = P.comp[c].fac[ua];
            const FactorPlan& F = P.fac[fi];
            int i = loc[c][pa], j = loc[c][pb];
            if (i > j) std::swap(i, j);
            if (F.kind == FK_PWAVE) {
              r = kRelZero;
            } else {
              const int k = F.kind == FK_GAUSS ? 2 : F.kind == FK_EXP ? 1 : F.order;
              const int tri = i * k - i * (i - 1) / 2 + (j - i);
              r = (signed char)(H.q_off[fi] + tri);
            }
          }
        }
        H.rel[np * kMaxComp + c] = r;
      }
    }
  H.npairs = np;
  if (nq > 120) {
    err = "too many second-derivative entries";
    return false;
  }
  return true;
}

// The staged row of one event: w, log2 P, s, r, l, q, then the event's
// coordinates (loaded for the whole chunk at once).
int hess_row_len(const Plan& P, const HessPlan& H) {
  return 2 + P.nfree + P.ncomp + P.ncomp * P.nfree + H.nq + P.ndim;
}

std::string plan_describe(const Plan& P) {
  std::string s = "components=" + std::to_string(P.ncomp) + " K=" + std::to_string(P.K) +
                  " sig=" + plan_signature(P) + " precision=" +
                  (P.precision == UML_MIXED ? "mixed" : "fp64");
  for (int c = 0; c < P.ncomp; ++c) {
    s += "\n  component " + std::to_string(c) + ": fractions";
    for (int k = 0; k < P.comp[c].nfrac; ++k)
      s += std::string(" ") + (P.comp[c].frac_sign[k] > 0 ? "" : "1-") + "p" +
           std::to_string(P.comp[c].frac_par[k]);
    for (int j = 0; j < P.comp[c].nfac; ++j) {
      const FactorPlan& F = P.fac[P.comp[c].fac[j]];
      s += std::string(" ") + kind_letter(F.kind) + "(dim" + std::to_string(F.dim[0]);
      if (F.kind == FK_PWAVE) s += "," + std::to_string(F.dim[1]) + "," + std::to_string(F.dim[2]);
      s += ")";
    }
  }
  return s;
}

}  // namespace uml
