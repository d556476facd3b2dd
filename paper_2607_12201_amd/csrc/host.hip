// Host side of the C ABI: argument validation, collocation tables, work lists, buffer layouts
// and kernel orchestration.  No device allocation happens here after colloc_create returns:
// tables, workspace and state live in caller memory.
#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <new>
#include <vector>

#include "../../include/colloc.h"
#include "big.h"
#include "ipm.h"
#include "kernels.h"

using namespace cl;

namespace cl {
size_t ipm_eval_lds(const Shape& S, int nt);
int kkt_prepare_attrs(const Shape& S);
int static_scratch(double** out);
int ipm_prepare_attrs(const Shape& S);
size_t ipm_trial_lds(const Shape& S, int max_ls);
}

// ------------------------------------------------------------------------ collocation tables
// Right-Radau points: roots of P_K(x) - P_(K-1)(x) on [-1, 1] (x = 1 is one of them), found by
// bracketing on a fine grid, bisection and a Newton polish; tau = (x + 1) / 2.
static void legendre(int n, double x, double* p, double* dp) {
  double p0 = 1.0, p1 = x, d0 = 0.0, d1 = 1.0;
  if (n == 0) { *p = 1.0; *dp = 0.0; return; }
  for (int k = 1; k < n; ++k) {
    double p2 = ((2.0 * k + 1.0) * x * p1 - k * p0) / (k + 1.0);
    double d2 = ((2.0 * k + 1.0) * (p1 + x * d1) - k * d0) / (k + 1.0);
    p0 = p1; p1 = p2; d0 = d1; d1 = d2;
  }
  *p = p1;
  *dp = d1;
}
static double radau_q(int K, double x, double* dq) {
  double a, da, b, db;
  legendre(K, x, &a, &da);
  legendre(K - 1, x, &b, &db);
  if (dq) *dq = da - db;
  return a - b;
}
static void radau_nodes(int K, double* tau) {  // tau[0..K], tau[0] = 0, tau[K] = 1
  tau[0] = 0.0;
  int found = 0;
  const int G = 20000;
  double xl = -1.0, fl = radau_q(K, xl, nullptr);
  for (int g = 1; g <= G && found < K - 1; ++g) {
    double xr = -1.0 + 2.0 * g / G;
    if (xr >= 1.0 - 1e-9) break;
    double fr = radau_q(K, xr, nullptr);
    if (fl == 0.0 || fl * fr < 0.0) {
      double a = xl, b = xr, fa = fl;
      for (int it = 0; it < 200 && b - a > 1e-17; ++it) {
        double m = 0.5 * (a + b), fm = radau_q(K, m, nullptr);
        if (fa * fm <= 0.0) b = m;
        else { a = m; fa = fm; }
      }
      double x = 0.5 * (a + b), dq;
      for (int it = 0; it < 3; ++it) {
        double q = radau_q(K, x, &dq);
        if (dq != 0.0) x -= q / dq;
      }
      tau[1 + found++] = 0.5 * (x + 1.0);
    }
    xl = xr;
    fl = fr;
  }
  tau[K] = 1.0;
}
// a[j][k] = l_j'(tau_k) from barycentric weights (differentiation matrix).
static void diff_weights(int K, const double* t, double a[CL_KMAX + 1][CL_KMAX + 1]) {
  double lam[CL_KMAX + 1];
  for (int j = 0; j <= K; ++j) {
    double p = 1.0;
    for (int m = 0; m <= K; ++m)
      if (m != j) p *= t[j] - t[m];
    lam[j] = 1.0 / p;
  }
  for (int k = 0; k <= K; ++k) {
    double diag = 0.0;
    for (int j = 0; j <= K; ++j) {
      if (j == k) continue;
      double v = (lam[j] / lam[k]) / (t[k] - t[j]);
      a[j][k] = v;
      diag -= v;
    }
    a[k][k] = diag;
  }
}
static double lagrange_value(int K, const double* t, int j, double x) {
  double v = 1.0;
  for (int m = 0; m <= K; ++m)
    if (m != j) v *= (x - t[m]) / (t[j] - t[m]);
  return v;
}

// ------------------------------------------------------------------------ handle
struct TableImage {
  std::vector<char> bytes;
  size_t add(const void* src, size_t n) {
    size_t off = (bytes.size() + 255) & ~(size_t)255;
    bytes.resize(off + (n ? n : 1));
    if (n) memcpy(bytes.data() + off, src, n);
    return off;
  }
};

struct EvPair {
  int phase;
  hipEvent_t a, b;
};

struct colloc_problem {
  Shape S;
  int n_inst;
  int64_t n_elem, n_total, m_total, n_meas;
  std::vector<int> N;
  std::vector<int64_t> x_off, g_off, e0;
  HostPlan hp;
  int nchunk;
  TableImage img;
  // offsets of each table in the image
  size_t o_N, o_x, o_g, o_e0, o_ei, o_el, o_eh, o_mptr, o_msp, o_mw, o_mys, o_react, o_param,
      o_logk, o_spp, o_spr, o_spnu, o_rxs, o_rxnu, o_z0, o_lo, o_hi, o_crp, o_cri, o_crj, o_stp,
      o_sti, o_sts, o_rqp, o_rqr, o_rqt, o_pcp, o_pcr, o_fqp, o_fqs, o_fqo, o_frp, o_frq, o_fru, o_cfr, o_cft, o_cfnu, o_zsp, o_zsk, o_zst, o_ztc, o_ctp,
      o_cts, o_ctr, o_ctnu;
  int cr_items_max;
  Tab tab;
  bool uploaded;
  // timing
  bool timing;
  std::vector<EvPair> evs;
  std::vector<hipEvent_t> pool;
  size_t pool_used;
  int open_phase[COLLOC_N_PHASES];
  hipEvent_t open_ev[COLLOC_N_PHASES];
  double ms[COLLOC_N_PHASES];
  int64_t launches[COLLOC_N_PHASES];
};

static hipEvent_t pool_get(colloc_problem* p) {
  if (p->pool_used == p->pool.size()) {
    hipEvent_t e;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    p->pool.push_back(e);
  }
  return p->pool[p->pool_used++];
}

static void phase_hook(void* ctx, int phase, int begin, hipStream_t st) {
  colloc_problem* p = (colloc_problem*)ctx;
  if (!p->timing || phase < 0 || phase >= COLLOC_N_PHASES) return;
  if (begin) {
    hipEvent_t e = pool_get(p);
    if (!e) return;
    (void)hipEventRecord(e, st);
    p->open_ev[phase] = e;
    p->open_phase[phase] = 1;
  } else if (p->open_phase[phase]) {
    hipEvent_t e = pool_get(p);
    if (!e) return;
    (void)hipEventRecord(e, st);
    p->evs.push_back({phase, p->open_ev[phase], e});
    p->open_phase[phase] = 0;
    p->launches[phase] += 1;
  }
}

#define CHECK(cond) \
  do {              \
    if (!(cond)) return COLLOC_EINVAL; \
  } while (0)

static size_t lds_limit() { return 160 * 1024; }

extern "C" int colloc_create(const colloc_instance_desc* inst, int32_t n_inst, int32_t K,
                             colloc_problem** out) {
  CHECK(out && inst && n_inst >= 1 && K >= 1 && K <= CL_KMAX);
  *out = nullptr;
  const int ns = inst[0].n_s, nr = inst[0].n_r, np = inst[0].n_p;
  CHECK(ns >= 1 && nr >= 0 && np >= 0 && np <= 4096 && ns <= 4096);
  for (int q = 0; q < n_inst; ++q) {
    const colloc_instance_desc& d = inst[q];
    CHECK(d.n_s == ns && d.n_r == nr && d.n_p == np && d.N >= 1);
    CHECK(nr == 0 || (d.react && d.prod && d.param && d.logk_fixed));
    CHECK(d.h && d.z0 && (np == 0 || (d.theta_lo && d.theta_hi)));
    CHECK(d.n_meas >= 0);
    CHECK(d.n_meas == 0 || (d.meas_elem && d.meas_species && d.meas_tau && d.meas_y && d.meas_sigma));
    for (int r = 0; r < nr; ++r) {
      for (int t = 0; t < 2; ++t) {
        CHECK(d.react[2 * r + t] >= -1 && d.react[2 * r + t] < ns);
        CHECK(d.prod[2 * r + t] >= -1 && d.prod[2 * r + t] < ns);
      }
      CHECK(d.param[r] >= -1 && d.param[r] < np);
      CHECK(isfinite(d.logk_fixed[r]));
    }
    for (int i = 0; i < d.N; ++i) CHECK(d.h[i] > 0.0 && isfinite(d.h[i]));
    for (int s = 0; s < ns; ++s) CHECK(isfinite(d.z0[s]));
    for (int c = 0; c < np; ++c) CHECK(d.theta_lo[c] < d.theta_hi[c]);
    for (int m = 0; m < d.n_meas; ++m) {
      CHECK(d.meas_elem[m] >= 0 && d.meas_elem[m] < d.N);
      CHECK(d.meas_species[m] >= 0 && d.meas_species[m] < ns);
      CHECK(d.meas_tau[m] >= 0.0 && d.meas_tau[m] <= 1.0);
      CHECK(d.meas_sigma[m] > 0.0 && isfinite(d.meas_y[m]));
    }
  }
  colloc_problem* p = new (std::nothrow) colloc_problem();
  if (!p) return COLLOC_ENOMEM;
  Shape& S = p->S;
  memset(&S, 0, sizeof(S));
  S.ns = ns; S.nr = nr; S.np = np; S.K = K;
  S.b = (K + 1) * ns;
  S.mI = K * ns;
  S.R = S.mI + 2 * ns + np;
  S.Rt = 2 * ns + np;
  double tau[CL_KMAX + 1];
  radau_nodes(K, tau);
  diff_weights(K, tau, S.a);
  // Factorization path: register-resident element blocks where they fit, otherwise (or when
  // COLLOC_FACTOR_PATH=tiled asks for it) the tiled matrix-core path.
  {
    const char* fp = getenv("COLLOC_FACTOR_PATH");
    const bool force_tiled = fp && strcmp(fp, "tiled") == 0;
    const bool force_reg = fp && strcmp(fp, "register") == 0;
    S.big = (force_tiled || !level0r_supported(S)) ? 1 : 0;
    if (force_reg && S.big) {
      delete p;
      return COLLOC_EUNSUPPORTED;
    }
  }
  // LDS budgets of the kernels (bytes); the tiled path's element assembly is checked once the
  // column lists are known
  int nt = elem_threads(S);
  size_t need = ipm_eval_lds(S, nt);
  size_t need_b = 0;
  if (!S.big) {
    need = std::max<size_t>(need, level0_lds_bytes(S, 0));
    need = std::max<size_t>(need, level0r_lds_bytes(S));
    need = std::max<size_t>(need, std::max(chain_lds_bytes(S, 1), chain_lds_bytes(S, 2)));
    need_b = sizeof(double) * std::max<size_t>(
        (size_t)2 * ns * ns + 2 * (size_t)ns * np + (size_t)np * np + 8,
        (size_t)7 * ns * ns + 3 * (size_t)ns * np + 8);
    need_b = std::max<size_t>(need_b, sizeof(double) * ((size_t)ns * ns + ns + np + (size_t)np * np + 1024));
    need_b = std::max<size_t>(need_b, sep_solve_lds(S));
    need_b = std::max<size_t>(need_b, border_solve_lds(S));
  } else {
    need_b = big_solve_lds(S);
  }
  // line-search trials: vectors, rate constants of every candidate, partial sums
  const size_t need_t = ipm_trial_lds(S, CL_MAX_LS);
  if (need > lds_limit() || need_b > lds_limit() || need_t > lds_limit() || nr * K > 65536) {
    delete p;
    return COLLOC_EUNSUPPORTED;
  }
  p->n_inst = n_inst;
  p->N.resize(n_inst);
  p->x_off.resize(n_inst);
  p->g_off.resize(n_inst);
  p->e0.resize(n_inst);
  int64_t xo = 0, go = 0, eo = 0, mo = 0;
  int maxN = 0;
  for (int q = 0; q < n_inst; ++q) {
    p->N[q] = inst[q].N;
    p->x_off[q] = xo;
    p->g_off[q] = go;
    p->e0[q] = eo;
    xo += (int64_t)inst[q].N * S.b + np;
    go += (int64_t)inst[q].N * S.b;
    eo += inst[q].N;
    mo += inst[q].n_meas;
    maxN = std::max(maxN, inst[q].N);
  }
  p->n_total = xo;
  p->m_total = go;
  p->n_elem = eo;
  p->n_meas = mo;
  if (eo > 0x7fffffff) { delete p; return COLLOC_EUNSUPPORTED; }
  // elements and measurements (CSR by element, in the instance's order within an element)
  std::vector<int> ei(eo), el(eo), mptr(eo + 1, 0), msp;
  std::vector<double> eh(eo), mw, mys;
  {
    std::vector<std::vector<int>> by(eo);
    for (int q = 0; q < n_inst; ++q)
      for (int i = 0; i < inst[q].N; ++i) {
        ei[p->e0[q] + i] = q;
        el[p->e0[q] + i] = i;
        eh[p->e0[q] + i] = inst[q].h[i];
      }
    for (int q = 0; q < n_inst; ++q)
      for (int m = 0; m < inst[q].n_meas; ++m) by[p->e0[q] + inst[q].meas_elem[m]].push_back(q * 0 + m);
    for (int64_t e = 0; e < eo; ++e) {
      int q = ei[e];
      const colloc_instance_desc& d = inst[q];
      for (int m : by[e]) {
        msp.push_back(d.meas_species[m]);
        for (int j = 0; j <= K; ++j) mw.push_back(lagrange_value(K, tau, j, d.meas_tau[m]) / d.meas_sigma[m]);
        mys.push_back(d.meas_y[m] / d.meas_sigma[m]);
      }
      mptr[e + 1] = mptr[e] + (int)by[e].size();
    }
  }
  // reaction tables
  std::vector<int> react((size_t)n_inst * nr * 2), param((size_t)n_inst * nr), spp((size_t)n_inst * (ns + 1)),
      spr, rxs((size_t)n_inst * nr * 4, -1);
  std::vector<int> rqp((size_t)n_inst * (ns + 1)), rqr, rqt, pcp((size_t)n_inst * (np + 1)), pcr;
  std::vector<double> logk((size_t)n_inst * nr), spnu, rxnu((size_t)n_inst * nr * 4, 0.0), z0((size_t)n_inst * ns),
      lo((size_t)n_inst * np), hi((size_t)n_inst * np);
  for (int q = 0; q < n_inst; ++q) {
    const colloc_instance_desc& d = inst[q];
    std::vector<double> nu((size_t)ns * nr, 0.0);
    for (int r = 0; r < nr; ++r) {
      for (int t = 0; t < 2; ++t) {
        react[((size_t)q * nr + r) * 2 + t] = d.react[2 * r + t];
        if (d.prod[2 * r + t] >= 0) nu[(size_t)d.prod[2 * r + t] * nr + r] += 1.0;
        if (d.react[2 * r + t] >= 0) nu[(size_t)d.react[2 * r + t] * nr + r] -= 1.0;
      }
      param[(size_t)q * nr + r] = d.param[r];
      logk[(size_t)q * nr + r] = d.logk_fixed[r];
      int k = 0;
      for (int s = 0; s < ns; ++s)
        if (nu[(size_t)s * nr + r] != 0.0) {
          if (k >= 4) { delete p; return COLLOC_EINVAL; }
          rxs[((size_t)q * nr + r) * 4 + k] = s;
          rxnu[((size_t)q * nr + r) * 4 + k] = nu[(size_t)s * nr + r];
          ++k;
        }
    }
    for (int s = 0; s < ns; ++s) {
      spp[(size_t)q * (ns + 1) + s] = (int)spr.size();
      for (int r = 0; r < nr; ++r)
        if (nu[(size_t)s * nr + r] != 0.0) {
          spr.push_back(r);
          spnu.push_back(nu[(size_t)s * nr + r]);
        }
    }
    spp[(size_t)q * (ns + 1) + ns] = (int)spr.size();
    for (int sp = 0; sp < ns; ++sp) {
      rqp[(size_t)q * (ns + 1) + sp] = (int)rqr.size();
      for (int r = 0; r < nr; ++r)
        for (int t = 0; t < 2; ++t)
          if (d.react[2 * r + t] == sp) {
            rqr.push_back(r);
            rqt.push_back(t);
          }
    }
    rqp[(size_t)q * (ns + 1) + ns] = (int)rqr.size();
    for (int c = 0; c < np; ++c) {
      pcp[(size_t)q * (np + 1) + c] = (int)pcr.size();
      for (int r = 0; r < nr; ++r)
        if (d.param[r] == c) pcr.push_back(r);
    }
    pcp[(size_t)q * (np + 1) + np] = (int)pcr.size();
    for (int s = 0; s < ns; ++s) z0[(size_t)q * ns + s] = d.z0[s];
    for (int c = 0; c < np; ++c) {
      lo[(size_t)q * np + c] = d.theta_lo[c];
      hi[(size_t)q * np + c] = d.theta_hi[c];
    }
  }
  for (int q = 0; q < n_inst; ++q) {
    S.lsp = std::max(S.lsp, spp[(size_t)q * (ns + 1) + ns] - spp[(size_t)q * (ns + 1)]);
    S.lrq = std::max(S.lrq, rqp[(size_t)q * (ns + 1) + ns] - rqp[(size_t)q * (ns + 1)]);
    S.lpc = std::max(S.lpc, pcp[(size_t)q * (np + 1) + np] - pcp[(size_t)q * (np + 1)]);
  }
  for (int64_t e = 0; e < eo; ++e) S.mmax = std::max(S.mmax, mptr[e + 1] - mptr[e]);
  // Pattern of F (tiled assembly): the terms of column u are every (reaction, slot) with u in the
  // slot and every species s the reaction changes; grouped by s (ascending, terms in reaction
  // order) they form the column's nonzeros (pairs).  Fth: for parameter c, every reaction of c
  // and every species it changes.
  std::vector<int> fqp((size_t)n_inst * (ns + 1)), fqs, fqo, frp((size_t)n_inst * (ns + 1)), frq, fru;
  std::vector<int> cfr, cft, ctp((size_t)n_inst * (np + 1)), cts, ctr, zsp((size_t)n_inst * (ns + 1)), zsk, zst, ztc;
  std::vector<double> cfnu, ctnu;
  for (int q = 0; q < n_inst; ++q) {
    const int* rs = rxs.data() + (size_t)q * nr * 4;
    const double* rn = rxnu.data() + (size_t)q * nr * 4;
    const int pair0 = (int)fqs.size();
    std::vector<std::vector<std::pair<int, int>>> rows(ns);   // per row s: (column u, pair)
    for (int u = 0; u < ns; ++u) {
      fqp[(size_t)q * (ns + 1) + u] = (int)fqs.size();
      struct Term { int s, r, t; double nu; };
      std::vector<Term> terms;
      for (int o = rqp[(size_t)q * (ns + 1) + u]; o < rqp[(size_t)q * (ns + 1) + u + 1]; ++o)
        for (int k = 0; k < 4; ++k)
          if (rs[rqr[o] * 4 + k] >= 0) terms.push_back({rs[rqr[o] * 4 + k], rqr[o], rqt[o], rn[rqr[o] * 4 + k]});
      std::stable_sort(terms.begin(), terms.end(), [](const Term& x, const Term& y) { return x.s < y.s; });
      for (size_t o = 0; o < terms.size(); ++o) {
        if (o == 0 || terms[o].s != terms[o - 1].s) {
          rows[terms[o].s].push_back({u, (int)fqs.size() - pair0});
          fqs.push_back(terms[o].s);
          fqo.push_back((int)cfr.size());
        }
        cfr.push_back(terms[o].r);
        cft.push_back(terms[o].t);
        cfnu.push_back(terms[o].nu);
      }
    }
    fqp[(size_t)q * (ns + 1) + ns] = (int)fqs.size();
    for (int s = 0; s < ns; ++s) {
      frp[(size_t)q * (ns + 1) + s] = (int)frq.size();
      for (const auto& uq : rows[s]) {
        fru.push_back(uq.first);
        frq.push_back(uq.second);
      }
    }
    frp[(size_t)q * (ns + 1) + ns] = (int)frq.size();
    for (int c = 0; c < np; ++c) {
      ctp[(size_t)q * (np + 1) + c] = (int)cts.size();
      for (int o = pcp[(size_t)q * (np + 1) + c]; o < pcp[(size_t)q * (np + 1) + c + 1]; ++o)
        for (int k = 0; k < 4; ++k)
          if (rs[pcr[o] * 4 + k] >= 0) {
            cts.push_back(rs[pcr[o] * 4 + k]);
            ctr.push_back(pcr[o]);
            ctnu.push_back(rn[pcr[o] * 4 + k]);
          }
    }
    ctp[(size_t)q * (np + 1) + np] = (int)cts.size();
    // Sparse terms of the z columns of species sp, grouped by the row they reach (key): the theta
    // rows of row sp of Fth (key ns + th, code = the ct entry), and for every reactant slot of sp
    // the other reactant's row at the column's node (key = that species, code -1 - (4 rr + 2 sl))
    // and the row of the reaction's parameter (key ns + th, code -2 - (4 rr + 2 sl)).
    const int c0 = ctp[(size_t)q * (np + 1)], zs0 = (int)zsk.size(), zt0 = (int)ztc.size();
    for (int sp = 0; sp < ns; ++sp) {
      struct Zt { int key, code; };
      std::vector<Zt> zt;
      for (int c = 0; c < np; ++c)
        for (int o = ctp[(size_t)q * (np + 1) + c]; o < ctp[(size_t)q * (np + 1) + c + 1]; ++o)
          if (cts[o] == sp) zt.push_back({ns + c, o - c0});
      for (int o = rqp[(size_t)q * (ns + 1) + sp]; o < rqp[(size_t)q * (ns + 1) + sp + 1]; ++o) {
        const int rr = rqr[o], sl = rqt[o], other = react[((size_t)q * nr + rr) * 2 + 1 - sl];
        if (other >= 0) zt.push_back({other, -1 - (4 * rr + 2 * sl)});
        if (param[(size_t)q * nr + rr] >= 0) zt.push_back({ns + param[(size_t)q * nr + rr], -2 - (4 * rr + 2 * sl)});
      }
      std::stable_sort(zt.begin(), zt.end(), [](const Zt& x, const Zt& y) { return x.key < y.key; });
      zsp[(size_t)q * (ns + 1) + sp] = (int)zsk.size();
      for (size_t i = 0; i < zt.size(); ++i) {
        if (i == 0 || zt[i].key != zt[i - 1].key) {
          zsk.push_back(zt[i].key);
          zst.push_back((int)ztc.size());
        }
        ztc.push_back(zt[i].code);
      }
    }
    zsp[(size_t)q * (ns + 1) + ns] = (int)zsk.size();
    S.lzs = std::max(S.lzs, (int)zsk.size() - zs0);
    S.lzt = std::max(S.lzt, (int)ztc.size() - zt0);
    S.lnf = std::max(S.lnf, fqp[(size_t)q * (ns + 1) + ns] - fqp[(size_t)q * (ns + 1)]);
    S.lct = std::max(S.lct, ctp[(size_t)q * (np + 1) + np] - ctp[(size_t)q * (np + 1)]);
  }
  if ((!S.big && level0r_lds_bytes(S) > lds_limit()) || (S.big && big_asm_lds(S) > lds_limit()) ||
      ipm_trial_lds(S, CL_MAX_LS) > lds_limit()) {   // sizes that depend on the list lengths
    delete p;
    return COLLOC_EUNSUPPORTED;
  }
  // cyclic-reduction work lists: separator j >= 1 is eliminated at level 1 + ctz(j)
  int L = 0;
  for (int q = 0; q < n_inst; ++q)
    if (p->N[q] > 1) L = std::max(L, 1 + (int)floor(log2((double)(p->N[q] - 1)) + 1e-12));
  if (L > 62) { delete p; return COLLOC_EUNSUPPORTED; }
  std::vector<int> crp(L + 1, 0), cri, crj;
  std::vector<int> stp(std::max(L, 1), 0), sti, sts;
  memset(&p->hp, 0, sizeof(p->hp));
  p->hp.L = L;
  for (int l = 1; l <= L; ++l) {
    int half = 1 << (l - 1);
    for (int q = 0; q < n_inst; ++q)
      for (int j = half; j < p->N[q]; j += 2 * half) {
        cri.push_back(q);
        crj.push_back(j);
      }
    crp[l] = (int)cri.size();
    p->hp.lvl[l] = crp[l] - crp[l - 1];
  }
  // step l = 1..L-1 touches every separator that is a multiple of 2^l (separator 0 included)
  for (int l = 1; l < L; ++l) {
    int step = 1 << l;
    for (int q = 0; q < n_inst; ++q)
      for (int s = 0; s < p->N[q]; s += step) {
        sti.push_back(q);
        sts.push_back(s);
      }
    stp[l] = (int)sti.size();
    p->hp.st[l] = stp[l] - stp[l - 1];
  }
  p->cr_items_max = 0;
  for (int l = 1; l <= L; ++l) p->cr_items_max = std::max(p->cr_items_max, p->hp.lvl[l]);
  p->nchunk = (int)std::max<int64_t>(1, cl_ceil_div(maxN, CL_THCHUNK));
  // pack
  TableImage& im = p->img;
  p->o_N = im.add(p->N.data(), sizeof(int) * n_inst);
  p->o_x = im.add(p->x_off.data(), sizeof(int64_t) * n_inst);
  p->o_g = im.add(p->g_off.data(), sizeof(int64_t) * n_inst);
  p->o_e0 = im.add(p->e0.data(), sizeof(int64_t) * n_inst);
  p->o_ei = im.add(ei.data(), sizeof(int) * eo);
  p->o_el = im.add(el.data(), sizeof(int) * eo);
  p->o_eh = im.add(eh.data(), sizeof(double) * eo);
  p->o_mptr = im.add(mptr.data(), sizeof(int) * (eo + 1));
  p->o_msp = im.add(msp.data(), sizeof(int) * msp.size());
  p->o_mw = im.add(mw.data(), sizeof(double) * mw.size());
  p->o_mys = im.add(mys.data(), sizeof(double) * mys.size());
  p->o_react = im.add(react.data(), sizeof(int) * react.size());
  p->o_param = im.add(param.data(), sizeof(int) * param.size());
  p->o_logk = im.add(logk.data(), sizeof(double) * logk.size());
  p->o_spp = im.add(spp.data(), sizeof(int) * spp.size());
  p->o_spr = im.add(spr.data(), sizeof(int) * spr.size());
  p->o_spnu = im.add(spnu.data(), sizeof(double) * spnu.size());
  p->o_rxs = im.add(rxs.data(), sizeof(int) * rxs.size());
  p->o_rqp = im.add(rqp.data(), sizeof(int) * rqp.size());
  p->o_rqr = im.add(rqr.data(), sizeof(int) * rqr.size());
  p->o_rqt = im.add(rqt.data(), sizeof(int) * rqt.size());
  p->o_pcp = im.add(pcp.data(), sizeof(int) * pcp.size());
  p->o_pcr = im.add(pcr.data(), sizeof(int) * pcr.size());
  p->o_rxnu = im.add(rxnu.data(), sizeof(double) * rxnu.size());
  p->o_z0 = im.add(z0.data(), sizeof(double) * z0.size());
  p->o_lo = im.add(lo.data(), sizeof(double) * lo.size());
  p->o_hi = im.add(hi.data(), sizeof(double) * hi.size());
  p->o_crp = im.add(crp.data(), sizeof(int) * crp.size());
  p->o_cri = im.add(cri.data(), sizeof(int) * cri.size());
  p->o_crj = im.add(crj.data(), sizeof(int) * crj.size());
  p->o_stp = im.add(stp.data(), sizeof(int) * stp.size());
  p->o_sti = im.add(sti.data(), sizeof(int) * sti.size());
  p->o_sts = im.add(sts.data(), sizeof(int) * sts.size());
  fqo.push_back((int)cfr.size());
  p->o_fqp = im.add(fqp.data(), sizeof(int) * fqp.size());
  p->o_fqs = im.add(fqs.data(), sizeof(int) * fqs.size());
  p->o_fqo = im.add(fqo.data(), sizeof(int) * fqo.size());
  p->o_frp = im.add(frp.data(), sizeof(int) * frp.size());
  p->o_frq = im.add(frq.data(), sizeof(int) * frq.size());
  p->o_fru = im.add(fru.data(), sizeof(int) * fru.size());
  p->o_cfr = im.add(cfr.data(), sizeof(int) * cfr.size());
  p->o_cft = im.add(cft.data(), sizeof(int) * cft.size());
  p->o_cfnu = im.add(cfnu.data(), sizeof(double) * cfnu.size());
  zst.push_back((int)ztc.size());
  p->o_zsp = im.add(zsp.data(), sizeof(int) * zsp.size());
  p->o_zsk = im.add(zsk.data(), sizeof(int) * zsk.size());
  p->o_zst = im.add(zst.data(), sizeof(int) * zst.size());
  p->o_ztc = im.add(ztc.data(), sizeof(int) * ztc.size());
  p->o_ctp = im.add(ctp.data(), sizeof(int) * ctp.size());
  p->o_cts = im.add(cts.data(), sizeof(int) * cts.size());
  p->o_ctr = im.add(ctr.data(), sizeof(int) * ctr.size());
  p->o_ctnu = im.add(ctnu.data(), sizeof(double) * ctnu.size());
  im.bytes.resize((im.bytes.size() + 255) & ~(size_t)255);
  p->uploaded = false;
  p->timing = false;
  p->pool_used = 0;
  memset(p->open_phase, 0, sizeof(p->open_phase));
  memset(p->ms, 0, sizeof(p->ms));
  memset(p->launches, 0, sizeof(p->launches));
  *out = p;
  return COLLOC_OK;
}

extern "C" int colloc_destroy(colloc_problem* p) {
  if (!p) return COLLOC_EINVAL;
  for (hipEvent_t e : p->pool) (void)hipEventDestroy(e);
  delete p;
  return COLLOC_OK;
}

extern "C" int colloc_layout_get(const colloc_problem* p, colloc_layout* out) {
  CHECK(p && out);
  out->n_inst = p->n_inst;
  out->n_s = p->S.ns;
  out->n_r = p->S.nr;
  out->n_p = p->S.np;
  out->K = p->S.K;
  out->b = p->S.b;
  out->n_elem = p->n_elem;
  out->n_total = p->n_total;
  out->m_total = p->m_total;
  out->jac_len = p->n_elem * p->S.K * p->S.nr * 3;
  out->hess_len = p->n_elem * p->S.K * p->S.nr * 4;
  out->x_off = p->x_off.data();
  out->g_off = p->g_off.data();
  out->elem_off = p->e0.data();
  out->N = p->N.data();
  return COLLOC_OK;
}

extern "C" size_t colloc_table_bytes(const colloc_problem* p) { return p ? p->img.bytes.size() : 0; }

extern "C" int colloc_upload(colloc_problem* p, void* table_dev, hipStream_t stream) {
  CHECK(p && table_dev && ((uintptr_t)table_dev % 256) == 0);
  hipError_t he = hipMemcpyAsync(table_dev, p->img.bytes.data(), p->img.bytes.size(),
                                 hipMemcpyHostToDevice, stream);
  if (he == hipSuccess) he = hipStreamSynchronize(stream);
  if (he != hipSuccess) {
    if (getenv("COLLOC_DEBUG")) fprintf(stderr, "colloc_upload: %s\n", hipGetErrorString(he));
    return COLLOC_EHIP;
  }
  char* b = (char*)table_dev;
  Tab& t = p->tab;
  int dev = 0, khz = 0;
  if (hipGetDevice(&dev) != hipSuccess ||
      hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, dev) != hipSuccess || khz <= 0)
    return COLLOC_EHIP;
  t.wclk_hz = 1e3 * (double)khz;
  t.n_inst = p->n_inst;
  t.L = p->hp.L;
  t.n_elem = p->n_elem;
  t.inst_N = (const int*)(b + p->o_N);
  t.inst_x = (const int64_t*)(b + p->o_x);
  t.inst_g = (const int64_t*)(b + p->o_g);
  t.inst_e0 = (const int64_t*)(b + p->o_e0);
  t.elem_inst = (const int*)(b + p->o_ei);
  t.elem_loc = (const int*)(b + p->o_el);
  t.elem_h = (const double*)(b + p->o_eh);
  t.elem_mptr = (const int*)(b + p->o_mptr);
  t.meas_sp = (const int*)(b + p->o_msp);
  t.meas_w = (const double*)(b + p->o_mw);
  t.meas_ys = (const double*)(b + p->o_mys);
  t.react = (const int*)(b + p->o_react);
  t.param = (const int*)(b + p->o_param);
  t.logk = (const double*)(b + p->o_logk);
  t.sp_ptr = (const int*)(b + p->o_spp);
  t.sp_r = (const int*)(b + p->o_spr);
  t.sp_nu = (const double*)(b + p->o_spnu);
  t.rx_sp = (const int*)(b + p->o_rxs);
  t.rq_ptr = (const int*)(b + p->o_rqp);
  t.rq_r = (const int*)(b + p->o_rqr);
  t.rq_t = (const int*)(b + p->o_rqt);
  t.pc_ptr = (const int*)(b + p->o_pcp);
  t.pc_r = (const int*)(b + p->o_pcr);
  t.rx_nu = (const double*)(b + p->o_rxnu);
  t.z0 = (const double*)(b + p->o_z0);
  t.th_lo = (const double*)(b + p->o_lo);
  t.th_hi = (const double*)(b + p->o_hi);
  t.cr_ptr = (const int*)(b + p->o_crp);
  t.cr_inst = (const int*)(b + p->o_cri);
  t.cr_j = (const int*)(b + p->o_crj);
  t.st_ptr = (const int*)(b + p->o_stp);
  t.st_inst = (const int*)(b + p->o_sti);
  t.st_s = (const int*)(b + p->o_sts);
  t.fq_ptr = (const int*)(b + p->o_fqp);
  t.fq_s = (const int*)(b + p->o_fqs);
  t.fq_o = (const int*)(b + p->o_fqo);
  t.fr_ptr = (const int*)(b + p->o_frp);
  t.fr_q = (const int*)(b + p->o_frq);
  t.fr_u = (const int*)(b + p->o_fru);
  t.cf_r = (const int*)(b + p->o_cfr);
  t.cf_t = (const int*)(b + p->o_cft);
  t.cf_nu = (const double*)(b + p->o_cfnu);
  t.zs_ptr = (const int*)(b + p->o_zsp);
  t.zs_key = (const int*)(b + p->o_zsk);
  t.zs_t = (const int*)(b + p->o_zst);
  t.zt_code = (const int*)(b + p->o_ztc);
  t.ct_ptr = (const int*)(b + p->o_ctp);
  t.ct_s = (const int*)(b + p->o_cts);
  t.ct_r = (const int*)(b + p->o_ctr);
  t.ct_nu = (const double*)(b + p->o_ctnu);
  t.cr_items_max = p->cr_items_max;
  if (ipm_prepare_attrs(p->S) != 0) return COLLOC_EHIP;
  if (p->S.big) {
    if (big_prepare_attrs(p->S) != 0) return COLLOC_EHIP;
  } else if (kkt_prepare_attrs(p->S) != 0 || level0_prepare_attrs(p->S) != 0) {
    return COLLOC_EHIP;
  }
  double* scr = nullptr;   // this device's static scratch of colloc_eval_noalloc
  if (static_scratch(&scr) != COLLOC_OK) return COLLOC_EHIP;
  p->uploaded = true;
  return COLLOC_OK;
}

// ------------------------------------------------------------------------ workspace layout
struct Carver {
  char* base;
  size_t off = 0;
  template <typename X>
  X* take(size_t count, size_t elem = sizeof(X)) {
    off = (off + 255) & ~(size_t)255;
    X* r = base ? (X*)(base + off) : nullptr;
    off += count * elem;
    return r;
  }
};

static Ws ws_layout(const colloc_problem* p, int prec, void* base, size_t* bytes) {
  const Shape& S = p->S;
  const size_t E = p->n_elem, I = p->n_inst;
  const size_t sz = prec ? 4 : 8;
  Carver c{(char*)base};
  Ws w;
  memset(&w, 0, sizeof(w));
  w.prec = prec;
  // precision-independent arrays first: their offsets are the same for both precisions
  w.jac = c.take<double>(E * S.K * S.nr * 3);
  w.hess = c.take<double>(E * S.K * S.nr * 4);
  w.Ds = c.take<double>(p->m_total);
  w.sxdw = c.take<double>(I * S.np);
  w.dw = c.take<double>(I);
  w.vtmp = c.take<double>(std::max<int64_t>(p->n_total, I));
  w.vtmp2 = c.take<double>(std::max<int64_t>(p->n_total, p->m_total));
  w.epart = c.take<double>(E * EP_N);
  w.ipart = c.take<double>(I * EP_N);
  w.flag = c.take<int>(I);
  w.irflag = c.take<int>(I);
  w.ircount = c.take<int>(I);
  w.runskip = c.take<int>(I);
  w.fbflag = c.take<int>(I);
  w.fbneed = c.take<int>(I);
  w.irpart = c.take<double>(E * 6);
  w.irnorm = c.take<double>(I * 2);
  w.rthp = c.take<double>(E * S.np);
  w.dcont = c.take<double>(E * S.ns);
  const bool big = S.big != 0;
  const size_t Er = big ? 0 : E;   // register-path block arrays (empty on the tiled path)
  w.ath = c.take<double>(E * S.np * S.np);
  w.thcr = c.take<double>(Er * S.np * S.np);
  w.S = c.take<double>(I * S.np * S.np);
  w.nchunk = p->nchunk;
  w.thred = c.take<double>(I * p->nchunk * S.np * S.np);
  w.thv = c.take<double>(I * p->nchunk * S.np);
  w.yI = c.take<double>(Er * S.mI);
  w.cS = c.take<double>(Er * S.ns);
  w.cP = c.take<double>(Er * S.ns);
  w.cB = c.take<double>(Er * S.np);
  w.ysep = c.take<double>(Er * S.ns);
  w.xsep = c.take<double>(E * S.ns);
  w.rcur = c.take<double>(E * S.ns);
  w.cBsep = c.take<double>(Er * S.np);
  w.xth = c.take<double>(I * S.np);
  if (big) {   // tiled path: FP64 vectors and border, then the blocks in the factor precision
    const BigGeom G = big_geom(S);
    w.evec = c.take<double>(E * G.Rp);
    w.svec = c.take<double>(E * G.Lp);
    w.bbuf = c.take<double>(I * G.Bp * G.Bp);
    w.linv = c.take<double>(E * 32 * 32);
    w.ebuf = c.take<char>(E * G.Rp * G.Rp, sz);
    w.sbuf = c.take<char>(E * G.Lp * G.Lp, sz);
  }
  // block data in the factor precision
  w.panel = c.take<char>(Er * S.R * S.mI, sz);
  w.dss = c.take<char>(Er * S.ns * S.ns, sz);
  w.bs = c.take<char>(Er * S.ns * S.np, sz);
  w.tprev = c.take<char>(Er * S.ns * S.ns, sz);
  w.e1 = c.take<char>(Er * S.ns * S.ns, sz);
  w.gprev = c.take<char>(Er * S.ns * S.np, sz);
  w.lsep = c.take<char>(Er * S.ns * S.ns, sz);
  w.ul = c.take<char>(Er * S.ns * S.ns, sz);
  w.ur = c.take<char>(Er * S.ns * S.ns, sz);
  w.ub = c.take<char>(Er * S.ns * S.np, sz);
  w.cTl = c.take<char>(Er * S.ns * S.ns, sz);
  w.cTr = c.take<char>(Er * S.ns * S.ns, sz);
  w.cE = c.take<char>(Er * S.ns * S.ns, sz);
  w.cGl = c.take<char>(Er * S.ns * S.np, sz);
  w.cGr = c.take<char>(Er * S.ns * S.np, sz);
  if (bytes) *bytes = (c.off + 255) & ~(size_t)255;
  return w;
}

static IpmState state_layout(const colloc_problem* p, void* base, size_t* bytes,
                             colloc_state_layout* lay) {
  const Shape& S = p->S;
  const size_t E = p->n_elem, I = p->n_inst, n = p->n_total, m = p->m_total;
  Carver c{(char*)base};
  IpmState s;
  auto rec = [&](double* ptr) { return (size_t)((char*)ptr - (char*)base); };
  (void)rec;
  size_t o;
  s.x = c.take<double>(n); o = c.off - n * 8; if (lay) lay->x = o;
  s.s = c.take<double>(m); o = c.off - m * 8; if (lay) lay->s = o;
  s.y = c.take<double>(m); o = c.off - m * 8; if (lay) lay->y = o;
  s.vL = c.take<double>(m); o = c.off - m * 8; if (lay) lay->vL = o;
  s.vU = c.take<double>(m); o = c.off - m * 8; if (lay) lay->vU = o;
  s.zL = c.take<double>(I * S.np); o = c.off - I * S.np * 8; if (lay) lay->zL = o;
  s.zU = c.take<double>(I * S.np); o = c.off - I * S.np * 8; if (lay) lay->zU = o;
  s.dx = c.take<double>(n); o = c.off - n * 8; if (lay) lay->dx = o;
  s.ds = c.take<double>(m); o = c.off - m * 8; if (lay) lay->ds = o;
  s.dy = c.take<double>(m); o = c.off - m * 8; if (lay) lay->dy = o;
  s.dvL = c.take<double>(m);
  s.dvU = c.take<double>(m);
  s.dzL = c.take<double>(I * S.np);
  s.dzU = c.take<double>(I * S.np);
  s.g = c.take<double>(m);
  s.grad = c.take<double>(n);
  s.rhs = c.take<double>(n);
  s.fth = c.take<double>(I * CL_FILTER_CAP);
  o = c.off - I * CL_FILTER_CAP * 8;
  if (lay) lay->fth = o;
  s.fph = c.take<double>(I * CL_FILTER_CAP);
  o = c.off - I * CL_FILTER_CAP * 8;
  if (lay) lay->fph = o;
  s.tpart = c.take<double>(E * CL_MAX_LS * 3);
  s.info = c.take<colloc_ipm_info>(I);
  o = c.off - I * sizeof(colloc_ipm_info);
  if (lay) lay->info = o;
  if (bytes) *bytes = (c.off + 255) & ~(size_t)255;
  return s;
}

extern "C" size_t colloc_workspace_bytes(const colloc_problem* p, int32_t precision) {
  if (!p || (precision != COLLOC_FP64 && precision != COLLOC_FP32_IR)) return 0;
  size_t b = 0;
  ws_layout(p, COLLOC_FP64, nullptr, &b);   // FP32_IR keeps room for its FP64 fallback
  return b;
}

extern "C" size_t colloc_state_bytes(const colloc_problem* p) {
  if (!p) return 0;
  size_t b = 0;
  state_layout(p, nullptr, &b, nullptr);
  return b;
}

extern "C" int colloc_state_layout_get(const colloc_problem* p, colloc_state_layout* out) {
  CHECK(p && out);
  char dummy_base[1];
  (void)dummy_base;
  size_t b = 0;
  // offsets are computed relative to a null base
  state_layout(p, nullptr, &b, out);
  return COLLOC_OK;
}

static bool aligned8(const void* q) { return q && ((uintptr_t)q % 8) == 0; }


extern "C" int colloc_eval(const colloc_problem* p, const double* x, double* obj, double* g,
                           void* ws_dev, hipStream_t stream) {
  CHECK(p && p->uploaded && aligned8(x) && aligned8(obj) && aligned8(g) && ws_dev);
  Ws w = ws_layout(p, 0, ws_dev, nullptr);
  return launch_eval(p->S, p->tab, w, x, obj, g, stream) ? COLLOC_EHIP : COLLOC_OK;
}

extern "C" int colloc_eval_noalloc(const colloc_problem* p, const double* x, double* obj, double* g,
                                   hipStream_t stream) {
  CHECK(p && p->uploaded && aligned8(x) && aligned8(obj) && aligned8(g));
  static_assert(EP_N == 13, "COLLOC_NOALLOC_MAX_ELEMS assumes 13 partial slots per element");
  if (p->n_elem > COLLOC_NOALLOC_MAX_ELEMS) {
    if (getenv("COLLOC_DEBUG"))
      fprintf(stderr, "colloc_eval_noalloc: %lld elements exceed the static scratch (%d)\n",
              (long long)p->n_elem, COLLOC_NOALLOC_MAX_ELEMS);
    return COLLOC_EINVAL;
  }
  double* scr = nullptr;
  if (static_scratch(&scr) != COLLOC_OK) return COLLOC_EHIP;
  Ws w;
  memset(&w, 0, sizeof(w));
  w.epart = scr;   // the only workspace array the evaluation kernels touch
  return launch_eval(p->S, p->tab, w, x, obj, g, stream) ? COLLOC_EHIP : COLLOC_OK;
}

extern "C" int colloc_derivs(const colloc_problem* p, const double* x, const double* y,
                             double* grad, double* jac, double* hess, hipStream_t stream) {
  CHECK(p && p->uploaded && aligned8(x) && aligned8(y) && aligned8(grad) && aligned8(jac) && aligned8(hess));
  return launch_derivs(p->S, p->tab, x, y, grad, jac, hess, stream) ? COLLOC_EHIP : COLLOC_OK;
}

static bool prec_ok(int32_t q) { return q == COLLOC_FP64 || q == COLLOC_FP32_IR; }

extern "C" int kkt_assemble(const colloc_problem* p, const double* jac, const double* hess,
                            const double* sigma_x, const double* sigma_s, const double* delta_w,
                            const double* r_x, const double* r_s, const double* r_y, void* ws_dev,
                            int32_t precision, double* rhs, hipStream_t stream) {
  CHECK(p && p->uploaded && aligned8(jac) && aligned8(hess) && aligned8(sigma_s) && aligned8(delta_w));
  CHECK(aligned8(r_x) && aligned8(r_s) && aligned8(r_y) && aligned8(rhs) && ws_dev && prec_ok(precision));
  CHECK(p->S.np == 0 || aligned8(sigma_x));
  Ws w = ws_layout(p, precision, ws_dev, nullptr);
  return launch_assemble(p->S, p->tab, w, jac, hess, sigma_x, sigma_s, delta_w, r_x, r_s, r_y, rhs,
                         stream)
             ? COLLOC_EHIP
             : COLLOC_OK;
}

extern "C" int kkt_factor(const colloc_problem* p, void* ws_dev, int32_t precision, int32_t* info,
                          hipStream_t stream) {
  CHECK(p && p->uploaded && ws_dev && info);
  CHECK(prec_ok(precision));
  Ws w = ws_layout(p, precision, ws_dev, nullptr);
  colloc_problem* pm = const_cast<colloc_problem*>(p);
  if (launch_factor(p->S, p->tab, p->hp, w, precision, false, phase_hook, pm, stream)) return COLLOC_EHIP;
  return launch_copy_flags(p->tab, w, info, stream) ? COLLOC_EHIP : COLLOC_OK;
}

extern "C" int kkt_solve(const colloc_problem* p, void* ws_dev, int32_t precision, const double* rhs,
                         double* dx, int32_t ir_max, double ir_tol, int32_t* ir_sweeps,
                         hipStream_t stream) {
  CHECK(p && p->uploaded && ws_dev && aligned8(rhs) && aligned8(dx) && ir_max >= 0 && prec_ok(precision));
  CHECK(rhs != dx && ir_tol >= 0.0 && ir_max <= 1000);
  Ws w = ws_layout(p, precision, ws_dev, nullptr);
  colloc_problem* pm = const_cast<colloc_problem*>(p);
  if (launch_solve_p(p->S, p->tab, p->hp, w, rhs, nullptr, dx, phase_hook, pm, stream)) return COLLOC_EHIP;
  if (launch_refine(p->S, p->tab, p->hp, w, rhs, dx, ir_max, ir_tol, phase_hook, pm, stream))
    return COLLOC_EHIP;
  if (ir_sweeps && launch_refine_report(p->tab, w, ir_sweeps, stream)) return COLLOC_EHIP;
  return COLLOC_OK;
}

extern "C" int kkt_matvec(const colloc_problem* p, void* ws_dev, const double* v, double* out,
                          hipStream_t stream) {
  CHECK(p && p->uploaded && ws_dev && aligned8(v) && aligned8(out) && v != out);
  Ws w = ws_layout(p, COLLOC_FP64, ws_dev, nullptr);
  return launch_matvec(p->S, p->tab, w, v, out, stream) ? COLLOC_EHIP : COLLOC_OK;
}

extern "C" void colloc_ipm_default_opts(colloc_ipm_opts* o) {
  if (!o) return;
  memset(o, 0, sizeof(*o));
  o->tol = 1e-6;
  o->acceptable_tol = 1e-4;
  o->acceptable_iter = 15;
  o->max_iter = 3000;
  o->mu_init = 0.1;
  o->tau_r = 1e-8;
  o->kappa_eps = 10.0;
  o->kappa_mu = 0.2;
  o->theta_mu = 1.5;
  o->tau_min = 0.99;
  o->kappa_sigma = 1e10;
  o->s_max = 100.0;
  o->bound_push = 1e-2;
  o->bound_frac = 1e-2;
  o->delta_w0 = 1e-4;
  o->delta_min = 1e-20;
  o->delta_max = 1e40;
  o->kappa_w_minus = 1.0 / 3.0;
  o->kappa_w_plus = 8.0;
  o->kappa_w_plus_bar = 100.0;
  o->gamma_theta = 1e-5;
  o->gamma_phi = 1e-8;
  o->s_theta = 1.1;
  o->s_phi = 2.3;
  o->eta_phi = 1e-8;
  o->delta_sw = 1.0;
  o->gamma_alpha = 0.05;
  o->max_ls = 40;
  o->precision = COLLOC_FP64;
  o->ir_max = 10;
  o->ir_tol = 1e-14;
  o->max_wall_s = 0.0;
}

static int check_opts(const colloc_ipm_opts* o) {
  if (!o) return 0;
  if (!(o->tol > 0 && o->tau_r > 0 && o->mu_init > 0 && o->max_ls >= 1 && o->max_ls <= CL_MAX_LS)) return 0;
  if (o->precision != COLLOC_FP64 && o->precision != COLLOC_FP32_IR) return 0;
  if (o->ir_max < 0 || o->ir_max > 100 || !(o->ir_tol >= 0.0)) return 0;
  if (!(o->max_wall_s >= 0.0)) return 0;
  return 1;
}

extern "C" int ipm_init(const colloc_problem* p, const double* x0, void* state, void* ws_dev,
                        const colloc_ipm_opts* opts, hipStream_t stream) {
  CHECK(p && p->uploaded && aligned8(x0) && state && ws_dev && check_opts(opts));
  Ws w = ws_layout(p, opts->precision, ws_dev, nullptr);
  IpmState st = state_layout(p, state, nullptr, nullptr);
  return launch_ipm_init(p->S, p->tab, st, w, x0, *opts, stream) ? COLLOC_EHIP : COLLOC_OK;
}

extern "C" int colloc_forward_init(const colloc_problem* p, const double* theta_dev, double* x_dev,
                                   int32_t* status_dev, hipStream_t stream) {
  CHECK(p && p->uploaded && aligned8(theta_dev) && aligned8(x_dev) && status_dev);
  const int rc = launch_fwd_init(p->S, p->tab, theta_dev, x_dev, status_dev, stream);
  return rc == -2 ? COLLOC_EUNSUPPORTED : rc ? COLLOC_EHIP : COLLOC_OK;
}

extern "C" int ipm_step(const colloc_problem* p, void* state, void* ws_dev, const colloc_ipm_opts* opts,
                        hipStream_t stream) {
  CHECK(p && p->uploaded && state && ws_dev && check_opts(opts));
  Ws w = ws_layout(p, opts->precision, ws_dev, nullptr);
  Ws w64 = ws_layout(p, COLLOC_FP64, ws_dev, nullptr);
  IpmState st = state_layout(p, state, nullptr, nullptr);
  colloc_problem* pm = const_cast<colloc_problem*>(p);
  return launch_ipm_step(p->S, p->tab, p->hp, st, w, w64, *opts, phase_hook, pm, stream) ? COLLOC_EHIP
                                                                                          : COLLOC_OK;
}

struct colloc_graph {
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
};

extern "C" int ipm_graph_create(const colloc_problem* p, void* state, void* ws_dev,
                                const colloc_ipm_opts* opts, int32_t steps, hipStream_t stream,
                                colloc_graph** out) {
  CHECK(p && p->uploaded && state && ws_dev && check_opts(opts) && out && stream && steps >= 1 &&
        steps <= 64);
  *out = nullptr;
  Ws w = ws_layout(p, opts->precision, ws_dev, nullptr);
  Ws w64 = ws_layout(p, COLLOC_FP64, ws_dev, nullptr);
  IpmState st = state_layout(p, state, nullptr, nullptr);
  colloc_graph* g = new (std::nothrow) colloc_graph;
  if (!g) return COLLOC_ENOMEM;
  if (hipStreamBeginCapture(stream, hipStreamCaptureModeThreadLocal) != hipSuccess) {
    delete g;
    return COLLOC_EHIP;
  }
  int rc = 0;
  for (int s = 0; s < steps && !rc; ++s)
    rc = launch_ipm_step(p->S, p->tab, p->hp, st, w, w64, *opts, nullptr, nullptr, stream);
  hipGraph_t graph = nullptr;
  const hipError_t ec = hipStreamEndCapture(stream, &graph);
  if (rc || ec != hipSuccess || !graph) {
    if (graph) hipGraphDestroy(graph);
    delete g;
    return COLLOC_EHIP;
  }
  g->graph = graph;
  if (hipGraphInstantiate(&g->exec, graph, nullptr, nullptr, 0) != hipSuccess) {
    hipGraphDestroy(graph);
    delete g;
    return COLLOC_EHIP;
  }
  *out = g;
  return COLLOC_OK;
}

extern "C" int ipm_graph_launch(colloc_graph* g, hipStream_t stream) {
  CHECK(g && g->exec);
  return hipGraphLaunch(g->exec, stream) == hipSuccess ? COLLOC_OK : COLLOC_EHIP;
}

extern "C" int ipm_graph_destroy(colloc_graph* g) {
  if (!g) return COLLOC_OK;
  if (g->exec) hipGraphExecDestroy(g->exec);
  if (g->graph) hipGraphDestroy(g->graph);
  delete g;
  return COLLOC_OK;
}

extern "C" int colloc_tile_options(const colloc_problem* p, int32_t which, int32_t* ts, int32_t cap) {
  CHECK(p && which >= 0 && which <= 2 && cap >= 0 && (ts || cap == 0));
  if (p->S.big) {   // the tiled path has one fixed tiling
    if (cap > 0) ts[0] = 0;
    return 1;
  }
  int tmp[8];
  const int n = tile_options(p->S, which, tmp, 8);
  for (int i = 0; i < n && i < cap; ++i) ts[i] = tmp[i];
  return n;
}

extern "C" int colloc_tile_set(colloc_problem* p, int32_t which, int32_t ts) {
  CHECK(p && which >= 0 && which <= 2 && (p->S.big ? ts == 0 : tile_valid(p->S, which, ts)));
  p->hp.ts[which] = ts;
  return COLLOC_OK;
}

extern "C" int colloc_tile_get(const colloc_problem* p, int32_t which) {
  CHECK(p && which >= 0 && which <= 2);
  return p->hp.ts[which];
}

extern "C" int colloc_timing_enable(colloc_problem* p, int32_t enable) {
  CHECK(p);
  p->timing = enable != 0;
  return COLLOC_OK;
}

extern "C" int colloc_timing_read(colloc_problem* p, double* ms, int64_t* launches, int32_t n) {
  CHECK(p && n >= 0);
  for (const EvPair& e : p->evs) {
    if (hipEventSynchronize(e.b) != hipSuccess) return COLLOC_EHIP;
    float t = 0.0f;
    if (hipEventElapsedTime(&t, e.a, e.b) != hipSuccess) return COLLOC_EHIP;
    p->ms[e.phase] += t;
  }
  p->evs.clear();
  p->pool_used = 0;
  for (int i = 0; i < n && i < COLLOC_N_PHASES; ++i) {
    if (ms) ms[i] = p->ms[i];
    if (launches) launches[i] = p->launches[i];
  }
  memset(p->ms, 0, sizeof(p->ms));
  memset(p->launches, 0, sizeof(p->launches));
  return COLLOC_OK;
}

extern "C" int colloc_tables(int32_t K, double* tau, double* a) {
  CHECK(K >= 1 && K <= CL_KMAX && tau && a);
  double t[CL_KMAX + 1], aa[CL_KMAX + 1][CL_KMAX + 1];
  radau_nodes(K, t);
  diff_weights(K, t, aa);
  for (int j = 0; j <= K; ++j) {
    tau[j] = t[j];
    for (int k = 0; k <= K; ++k) a[j * (K + 1) + k] = aa[j][k];
  }
  return COLLOC_OK;
}
