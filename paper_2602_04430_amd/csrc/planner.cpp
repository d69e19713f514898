// Plan optimizer over profiled log-odds (host code).
//
// Section 4.1: a logical filter runs as a cascade of candidate physical operators; the
// choice of operators and their log-odds thresholds is relaxed (pick factor
// sigmoid(s / tau), soft decisions softmax([LO - theta+, theta- - LO, 0] / tau)) so that
// Eqs. 1-4 become differentiable; the loss of Eqs. 10-13 (normalised cost plus hinges on the
// Beta credible lower bounds of recall and precision, Eqs. 8-9) is minimised by Adam while
// tau falls exponentially, and the plan is read off at tau = 0.  Section 4.2: several
// filters are combined through the global result (a tuple passes iff every filter accepts
// it), and the selected physical operators are ordered by the subset dynamic programme of
// Algorithm 1.
//
// The gradient is exact reverse mode through the relaxed cascade; the derivative of a
// credible bound with respect to the Beta parameters follows from the implicit function
// theorem, dl/da = -(dI/da) / density(l), with dI/da by a central difference.
#include <algorithm>
#include <cmath>
#include <limits>
#include <string>
#include <vector>

#include "../../include/kvop.h"
#include "host_util.h"

using kvop::fail;

namespace {

// ------------------------------------------------------------------ incomplete beta

double log_beta(double a, double b) { return std::lgamma(a) + std::lgamma(b) - std::lgamma(a + b); }

// Continued fraction of the regularised incomplete beta function (the expansion of DLMF
// 8.17.22), evaluated by the modified Lentz method: I_x(a, b) = front / a * 1 / (1 + d1 /
// (1 + d2 / (1 + ...))), with d_{2m+1} = -(a+m)(a+b+m) x / ((a+2m)(a+2m+1)) and
// d_{2m} = m (b-m) x / ((a+2m-1)(a+2m)).
double beta_cf(double a, double b, double x) {
  const double tiny = 1e-300, eps = 1e-16;
  double f = 1.0, C = 1.0, D = 0.0;
  for (int n = 1; n <= 20000; n++) {
    int m = n / 2;
    double d;
    if (n & 1)
      d = -(a + m) * (a + b + m) * x / ((a + 2.0 * m) * (a + 2.0 * m + 1.0));
    else
      d = m * (b - m) * x / ((a + 2.0 * m - 1.0) * (a + 2.0 * m));
    D = 1.0 + d * D;
    if (std::fabs(D) < tiny) D = tiny;
    C = 1.0 + d / C;
    if (std::fabs(C) < tiny) C = tiny;
    D = 1.0 / D;
    double delta = C * D;
    f *= delta;
    if (std::fabs(delta - 1.0) < eps) break;
  }
  // the fraction above is 1 / (1 + d1 / (1 + ...)) once the leading 1 / (...) is applied
  return 1.0 / f;
}

double inc_beta(double a, double b, double x) {
  if (x <= 0.0) return 0.0;
  if (x >= 1.0) return 1.0;
  double front = std::exp(a * std::log(x) + b * std::log1p(-x) - log_beta(a, b));
  if (x < (a + 1.0) / (a + b + 2.0)) return front * beta_cf(a, b, x) / a;
  return 1.0 - front * beta_cf(b, a, 1.0 - x) / b;
}

// x with I_x(a, b) = p, by bisection (I is increasing in x) to full double resolution.
double inc_beta_inv(double a, double b, double p) {
  double lo = 0.0, hi = 1.0;
  for (int it = 0; it < 200 && hi - lo > 1e-17; it++) {
    double mid = 0.5 * (lo + hi);
    if (mid <= lo || mid >= hi) break;
    if (inc_beta(a, b, mid) < p)
      lo = mid;
    else
      hi = mid;
  }
  return 0.5 * (lo + hi);
}

// Lower bound l with P(X >= l) = alpha for X ~ Beta(a, b), and its partial derivatives.
struct Bound {
  double l, dl_da, dl_db;
};

Bound lower_bound(double a, double b, double alpha, bool with_grad) {
  Bound r{inc_beta_inv(a, b, 1.0 - alpha), 0.0, 0.0};
  if (!with_grad) return r;
  double x = r.l;
  if (x <= 0.0 || x >= 1.0) return r;
  double dens = std::exp((a - 1.0) * std::log(x) + (b - 1.0) * std::log1p(-x) - log_beta(a, b));
  if (!(dens > 0.0) || !std::isfinite(dens)) return r;
  double ha = 1e-5 * a, hb = 1e-5 * b;
  double dIa = (inc_beta(a + ha, b, x) - inc_beta(a - ha, b, x)) / (2.0 * ha);
  double dIb = (inc_beta(a, b + hb, x) - inc_beta(a, b - hb, x)) / (2.0 * hb);
  r.dl_da = -dIa / dens;
  r.dl_db = -dIb / dens;
  return r;
}

// ------------------------------------------------------------------ problem checks

struct Layout {
  std::vector<int> first;  // first operator index of every filter
  int total = 0;
};

kvop_status check_problem(const kvop_plan_problem* pb, Layout& lay) {
  if (!pb || pb->n_filters < 1 || pb->n_filters > 64 || !pb->n_ops || !pb->cost || !pb->log_odds || !pb->gold ||
      pb->n_tuples < 1)
    return fail(KVOP_EINVAL, "bad plan problem");
  if (!(pb->alpha > 0.0 && pb->alpha < 1.0)) return fail(KVOP_EINVAL, "alpha must be in (0, 1)");
  if (!(pb->target_recall >= 0.0 && pb->target_recall <= 1.0 && pb->target_precision >= 0.0 &&
        pb->target_precision <= 1.0))
    return fail(KVOP_EINVAL, "targets must be in [0, 1]");
  lay.first.assign(pb->n_filters + 1, 0);
  for (int j = 0; j < pb->n_filters; j++) {
    if (pb->n_ops[j] < 1 || pb->n_ops[j] > 64) return fail(KVOP_EINVAL, "every filter needs 1..64 operators");
    lay.first[j + 1] = lay.first[j] + pb->n_ops[j];
  }
  lay.total = lay.first[pb->n_filters];
  for (int i = 0; i < lay.total; i++)
    if (!(pb->cost[i] > 0.0) || !std::isfinite(pb->cost[i])) return fail(KVOP_EINVAL, "costs must be positive");
  for (int64_t k = 0; k < (int64_t)lay.total * pb->n_tuples; k++)
    if (!std::isfinite(pb->log_odds[k])) return fail(KVOP_EINVAL, "non-finite log-odds");
  return KVOP_OK;
}

inline double sigmoid(double x) {
  if (x >= 0) return 1.0 / (1.0 + std::exp(-x));
  double e = std::exp(x);
  return e / (1.0 + e);
}

// ------------------------------------------------------------------ relaxed loss and gradient

struct LossParts {
  double loss, cost_term, tp, fp, fn, recall_lb, precision_lb;
};

// params: per operator (s, theta+, theta-), filters in order.  grad may be null.
LossParts relaxed_loss(const kvop_plan_problem* pb, const Layout& lay, const double* params, double tau, double beta,
                       double* grad) {
  const int S = pb->n_tuples, F = pb->n_filters;
  double csum = 0.0;
  for (int i = 0; i < lay.total; i++) csum += pb->cost[i];
  // forward: per filter the soft accept of every tuple, per tuple the relaxed cost
  std::vector<double> acc((size_t)F * S), sig(lay.total);
  double cost_total = 0.0;
  for (int i = 0; i < lay.total; i++) sig[i] = sigmoid(params[3 * i] / tau);
  for (int j = 0; j < F; j++) {
    for (int t = 0; t < S; t++) {
      double a = 0.0, u = 1.0;
      for (int i = lay.first[j]; i < lay.first[j + 1]; i++) {
        double lo = pb->log_odds[(int64_t)i * S + t];
        double z0 = (lo - params[3 * i + 1]) / tau, z1 = (params[3 * i + 2] - lo) / tau;
        double mx = std::max(std::max(z0, z1), 0.0);
        double e0 = std::exp(z0 - mx), e1 = std::exp(z1 - mx), e2 = std::exp(-mx), den = e0 + e1 + e2;
        double pa = e0 / den, pr = e1 / den;
        cost_total += u * sig[i] * pb->cost[i];
        a += u * sig[i] * pa;
        u *= 1.0 - sig[i] * (pa + pr);
      }
      acc[(size_t)j * S + t] = a;
    }
  }
  std::vector<double> A(S, 1.0);
  std::vector<int> G(S, 1);
  for (int j = 0; j < F; j++)
    for (int t = 0; t < S; t++) {
      A[t] *= acc[(size_t)j * S + t];
      G[t] &= pb->gold[(int64_t)j * S + t] == 1;
    }
  double TP = 0, FP = 0, FN = 0;
  for (int t = 0; t < S; t++) {
    TP += A[t] * G[t];
    FP += A[t] * (1 - G[t]);
    FN += (1.0 - A[t]) * G[t];
  }
  bool g = grad != nullptr;
  Bound br = lower_bound(1.0 + TP, 1.0 + FN, pb->alpha, g);
  Bound bp = lower_bound(1.0 + TP, 1.0 + FP, pb->alpha, g);
  double w = 1.0 / ((double)S * csum);
  LossParts out;
  out.cost_term = cost_total * w;
  out.tp = TP, out.fp = FP, out.fn = FN, out.recall_lb = br.l, out.precision_lb = bp.l;
  bool rec_on = pb->target_recall - br.l > 0.0, prec_on = pb->target_precision - bp.l > 0.0;
  out.loss = out.cost_term + beta * (prec_on ? pb->target_precision - bp.l : 0.0) +
             beta * (rec_on ? pb->target_recall - br.l : 0.0);
  if (!g) return out;
  // dL/dTP, dL/dFP, dL/dFN through the active hinges
  double gTP = 0, gFP = 0, gFN = 0;
  if (rec_on) gTP -= beta * br.dl_da, gFN -= beta * br.dl_db;
  if (prec_on) gTP -= beta * bp.dl_da, gFP -= beta * bp.dl_db;
  std::fill(grad, grad + 3 * lay.total, 0.0);
  std::vector<double> ua(64), pa_(64), pr_(64);
  for (int j = 0; j < F; j++) {
    for (int t = 0; t < S; t++) {
      // dL/dA_t, then dL/d(accept of filter j) = dL/dA_t * prod of the other filters' accepts
      double gA = G[t] ? (gTP - gFN) : gFP;
      double other = 1.0;
      for (int k = 0; k < F; k++)
        if (k != j) other *= acc[(size_t)k * S + t];
      double ga = gA * other;  // dL/da_i for every i (a_i carries into a_n with weight 1)
      // recompute the forward values of this tuple's cascade
      int n = lay.first[j + 1] - lay.first[j];
      double u = 1.0;
      for (int q = 0; q < n; q++) {
        int i = lay.first[j] + q;
        double lo = pb->log_odds[(int64_t)i * S + t];
        double z0 = (lo - params[3 * i + 1]) / tau, z1 = (params[3 * i + 2] - lo) / tau;
        double mx = std::max(std::max(z0, z1), 0.0);
        double e0 = std::exp(z0 - mx), e1 = std::exp(z1 - mx), e2 = std::exp(-mx), den = e0 + e1 + e2;
        ua[q] = u, pa_[q] = e0 / den, pr_[q] = e1 / den;
        u *= 1.0 - sig[i] * (pa_[q] + pr_[q]);
      }
      double gu = 0.0;  // dL/du_q for the unsure value after operator q (none after the last)
      for (int q = n - 1; q >= 0; q--) {
        int i = lay.first[j] + q;
        double s = sig[i], pa = pa_[q], pr = pr_[q], up = ua[q], c = pb->cost[i] * w;
        // a_q = a_{q-1} + up s pa ; u_q = up (1 - s (pa + pr)) ; cost += up s c
        double g_sig = ga * up * pa - gu * up * (pa + pr) + up * c;
        double g_pa = ga * up * s - gu * up * s;
        double g_pr = -gu * up * s;
        // softmax over z = (z0, z1, 0) / tau: dL/dz_m = p_m (G_m - sum_k G_k p_k) / tau
        double mean = g_pa * pa + g_pr * pr;
        double g_z0 = pa * (g_pa - mean) / tau, g_z1 = pr * (g_pr - mean) / tau;
        grad[3 * i] += g_sig * s * (1.0 - s) / tau;
        grad[3 * i + 1] -= g_z0;
        grad[3 * i + 2] += g_z1;
        gu = ga * s * pa + gu * (1.0 - s * (pa + pr)) + s * c;
      }
    }
  }
  return out;
}

double temperature(int k, const kvop_plan_opts* o) {
  if (o->steps <= 1) return o->tau0;
  return o->tau0 * std::pow(o->tau_end / o->tau0, (double)k / (double)(o->steps - 1));
}

// ------------------------------------------------------------------ the discrete plan

struct HardEval {
  kvop_plan_report rep;
  std::vector<double> inter, intra;
  std::vector<int32_t> processed;
  std::vector<int8_t> accept;
};

HardEval hard_eval(const kvop_plan_problem* pb, const Layout& lay, const int8_t* sel, const float* tp,
                   const float* tn) {
  const int S = pb->n_tuples, F = pb->n_filters;
  HardEval h;
  h.inter.assign(lay.total, 0.0), h.intra.assign(lay.total, 0.0), h.processed.assign(lay.total, 0);
  h.accept.assign(S, 1);
  double csum = 0.0, total = 0.0;
  for (int i = 0; i < lay.total; i++) csum += pb->cost[i];
  std::vector<int8_t> acc(S), uns(S);
  for (int j = 0; j < F; j++) {
    std::fill(acc.begin(), acc.end(), 0);
    std::fill(uns.begin(), uns.end(), 1);
    for (int i = lay.first[j]; i < lay.first[j + 1]; i++) {
      int64_t n_not_rej = 0, n_uns = 0, n_proc = 0;
      for (int t = 0; t < S; t++) {
        float lo = pb->log_odds[(int64_t)i * S + t];
        int d = lo > tp[i] ? 1 : (lo < tn[i] ? 0 : -1);
        n_not_rej += d != 0;
        n_uns += d == -1;
        if (sel[i] && uns[t]) {
          n_proc++;
          if (d == 1) acc[t] = 1;
          if (d != -1) uns[t] = 0;
        }
      }
      h.inter[i] = (double)n_not_rej / S;
      h.intra[i] = (double)n_uns / S;
      h.processed[i] = (int32_t)n_proc;
      total += (double)n_proc * pb->cost[i];
    }
    for (int t = 0; t < S; t++) h.accept[t] &= acc[t];
  }
  double TP = 0, FP = 0, FN = 0;
  for (int t = 0; t < S; t++) {
    int gt = 1;
    for (int j = 0; j < F; j++) gt &= pb->gold[(int64_t)j * S + t] == 1;
    TP += h.accept[t] && gt;
    FP += h.accept[t] && !gt;
    FN += !h.accept[t] && gt;
  }
  h.rep.tp = TP, h.rep.fp = FP, h.rep.fn = FN;
  h.rep.recall_lb = lower_bound(1.0 + TP, 1.0 + FN, pb->alpha, false).l;
  h.rep.precision_lb = lower_bound(1.0 + TP, 1.0 + FP, pb->alpha, false).l;
  h.rep.cost_frac = total / ((double)S * csum);
  return h;
}

}  // namespace

// ------------------------------------------------------------------ C ABI

extern "C" {

kvop_status kvop_beta_lower_bound(double a, double b, double alpha, double* out) {
  if (!out || !(a > 0.0) || !(b > 0.0) || !std::isfinite(a) || !std::isfinite(b) || !(alpha > 0.0 && alpha < 1.0))
    return fail(KVOP_EINVAL, "need a, b > 0 and alpha in (0, 1)");
  *out = lower_bound(a, b, alpha, false).l;
  return KVOP_OK;
}

kvop_status kvop_plan_loss(const kvop_plan_problem* pb, const double* params, double tau, double beta,
                           double* loss_out, double* grad_out) {
  Layout lay;
  kvop_status s = check_problem(pb, lay);
  if (s != KVOP_OK) return s;
  if (!params || !loss_out || !(tau > 0.0) || !(beta >= 0.0)) return fail(KVOP_EINVAL, "bad loss arguments");
  *loss_out = relaxed_loss(pb, lay, params, tau, beta, grad_out).loss;
  return KVOP_OK;
}

kvop_status kvop_plan_optimize(const kvop_plan_problem* pb, const kvop_plan_opts* o, double* params_out,
                               int8_t* selected_out, float* theta_pos_out, float* theta_neg_out,
                               double* loss_trace_out, kvop_plan_report* report_out) {
  Layout lay;
  kvop_status st = check_problem(pb, lay);
  if (st != KVOP_OK) return st;
  if (!o || o->steps < 1 || !(o->lr > 0.0) || !(o->beta >= 0.0) || !(o->tau_end > 0.0) || !(o->tau0 >= o->tau_end) ||
      !std::isfinite(o->theta0))
    return fail(KVOP_EINVAL, "bad optimizer options");
  if (!selected_out || !theta_pos_out || !theta_neg_out) return fail(KVOP_EINVAL, "null output");
  const int P = 3 * lay.total;
  std::vector<double> p(P), g(P), m(P, 0.0), v(P, 0.0);
  for (int i = 0; i < lay.total; i++) p[3 * i] = 0.0, p[3 * i + 1] = o->theta0, p[3 * i + 2] = -o->theta0;
  const double b1 = 0.9, b2 = 0.999, eps = 1e-8;
  for (int k = 0; k < o->steps; k++) {
    double tau = temperature(k, o);
    LossParts lp = relaxed_loss(pb, lay, p.data(), tau, o->beta, g.data());
    if (loss_trace_out) loss_trace_out[k] = lp.loss;
    double c1 = 1.0 - std::pow(b1, k + 1), c2 = 1.0 - std::pow(b2, k + 1);
    for (int q = 0; q < P; q++) {
      m[q] = b1 * m[q] + (1.0 - b1) * g[q];
      v[q] = b2 * v[q] + (1.0 - b2) * g[q] * g[q];
      p[q] -= o->lr * (m[q] / c1) / (std::sqrt(v[q] / c2) + eps);
    }
  }
  // tau = 0: selected iff s > 0; crossed thresholds collapse to their midpoint
  for (int i = 0; i < lay.total; i++) {
    double tp = p[3 * i + 1], tn = p[3 * i + 2];
    selected_out[i] = p[3 * i] > 0.0;
    if (tp < tn) tp = tn = 0.5 * (tp + tn);
    theta_pos_out[i] = (float)tp;
    theta_neg_out[i] = (float)tn;
  }
  if (params_out) std::copy(p.begin(), p.end(), params_out);
  if (report_out) *report_out = hard_eval(pb, lay, selected_out, theta_pos_out, theta_neg_out).rep;
  return KVOP_OK;
}

kvop_status kvop_plan_evaluate(const kvop_plan_problem* pb, const int8_t* selected, const float* theta_pos,
                               const float* theta_neg, kvop_plan_report* report_out, double* sel_inter_out,
                               double* sel_intra_out, int32_t* processed_out, int8_t* accept_out) {
  Layout lay;
  kvop_status st = check_problem(pb, lay);
  if (st != KVOP_OK) return st;
  if (!selected || !theta_pos || !theta_neg) return fail(KVOP_EINVAL, "null plan");
  for (int i = 0; i < lay.total; i++)
    if (std::isnan(theta_pos[i]) || std::isnan(theta_neg[i])) return fail(KVOP_EINVAL, "NaN threshold");
  HardEval h = hard_eval(pb, lay, selected, theta_pos, theta_neg);
  if (report_out) *report_out = h.rep;
  if (sel_inter_out) std::copy(h.inter.begin(), h.inter.end(), sel_inter_out);
  if (sel_intra_out) std::copy(h.intra.begin(), h.intra.end(), sel_intra_out);
  if (processed_out) std::copy(h.processed.begin(), h.processed.end(), processed_out);
  if (accept_out) std::copy(h.accept.begin(), h.accept.end(), accept_out);
  return KVOP_OK;
}

kvop_status kvop_plan_reorder(int32_t n_ops, const int32_t* impl, const double* cost, const double* sel_inter,
                              const double* sel_intra, double n_tuples, int32_t* order_out, double* cost_out) {
  if (n_ops < 1 || n_ops > 20 || !impl || !cost || !sel_inter || !sel_intra || !order_out || !cost_out ||
      !(n_tuples >= 0.0))
    return fail(KVOP_EINVAL, "need 1..20 operators and non-null arrays");
  // logical operators renumbered densely (at most n_ops of them), so the table is
  // 2^n_ops x (distinct logical operators) pending counts
  int dense[64], n_log = 0;
  std::fill(dense, dense + 64, -1);
  std::vector<int> lid(n_ops);
  for (int i = 0; i < n_ops; i++) {
    if (impl[i] < 0 || impl[i] >= 64) return fail(KVOP_EINVAL, "logical operator index out of range");
    if (!(sel_inter[i] >= 0.0 && sel_inter[i] <= 1.0 && sel_intra[i] >= 0.0 && sel_intra[i] <= 1.0) ||
        !(cost[i] >= 0.0) || !std::isfinite(cost[i]))
      return fail(KVOP_EINVAL, "selectivities must be in [0, 1], costs finite and >= 0");
    if (dense[impl[i]] < 0) dense[impl[i]] = n_log++;
    lid[i] = dense[impl[i]];
  }
  const uint32_t full = (1u << n_ops) - 1u;
  const double inf = std::numeric_limits<double>::infinity();
  std::vector<double> best(full + 1, inf), rem((size_t)(full + 1) * n_log, 0.0);
  std::vector<int8_t> parent(full + 1, -1);
  best[0] = 0.0;
  for (int l = 0; l < n_log; l++) rem[l] = n_tuples;
  // subsets in increasing cardinality; popcount order is implied by visiting every subset
  // before any of its supersets, which ascending numeric order guarantees
  for (uint32_t S = 0; S < full; S++) {
    if (best[S] == inf) continue;
    const double* r = &rem[(size_t)S * n_log];
    for (int i = 0; i < n_ops; i++) {
      if (S >> i & 1u) continue;
      uint32_t T = S | (1u << i);
      double c = best[S] + cost[i] * r[lid[i]];
      if (c < best[T]) {
        best[T] = c;
        parent[T] = (int8_t)i;
        double* rt = &rem[(size_t)T * n_log];
        for (int l = 0; l < n_log; l++) rt[l] = r[l] * (l == lid[i] ? sel_intra[i] : sel_inter[i]);
      }
    }
  }
  uint32_t x = full;
  for (int k = n_ops - 1; k >= 0; k--) {
    int i = parent[x];
    order_out[k] = i;
    x &= ~(1u << i);
  }
  *cost_out = best[full];
  return KVOP_OK;
}

}  // extern "C"
