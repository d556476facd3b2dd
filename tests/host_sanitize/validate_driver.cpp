// Host-side checks of the C ABI, built with AddressSanitizer and UndefinedBehaviorSanitizer:
// colloc_create must reject malformed batches with COLLOC_EINVAL before it reads past any
// array it was given, and build the tables of valid batches (register and tiled factorization
// paths, several collocation orders, reactions sharing a parameter, bimolecular 2A reactions)
// without invalid memory accesses.  No call here touches a GPU.
#include <math.h>
#include <stdio.h>
#include <stdlib.h>

#include <vector>

#include "colloc.h"

static int failures = 0;
#define EXPECT(cond)                                                    \
  do {                                                                  \
    if (!(cond)) {                                                      \
      fprintf(stderr, "%s:%d: expectation failed: %s\n", __FILE__, __LINE__, #cond); \
      ++failures;                                                       \
    }                                                                   \
  } while (0)

// A synthetic mass-action network on ns species: a ring of conversions A_i -> A_(i+1), one
// bimolecular A_i + A_(i+1) -> A_(i+2) per species and one 2A_0 -> A_1; parameters shared by
// pairs of reactions; measurements of every other species at every element end.
struct Net {
  int ns, nr, np, N;
  std::vector<int32_t> react, prod, param, meas_elem, meas_sp;
  std::vector<double> logk, h, z0, tau, y, sigma, lo, hi;
  colloc_instance_desc d;
  Net(int ns_, int N_) : ns(ns_), N(N_) {
    for (int i = 0; i < ns; ++i) add(i, -1, (i + 1) % ns, -1);
    for (int i = 0; i < ns; ++i) add(i, (i + 1) % ns, (i + 2) % ns, -1);
    add(0, 0, 1, -1);
    nr = (int)param.size();
    np = (nr + 1) / 2;
    for (int r = 0; r < nr; ++r) param[r] = r / 2;   // two reactions per parameter
    param[nr - 1] = -1;                               // the last rate fixed
    for (int i = 0; i < N; ++i) h.push_back(0.1 + 0.01 * i);
    for (int s = 0; s < ns; ++s) z0.push_back(0.5 + 0.1 * s);
    for (int i = 0; i < N; ++i)
      for (int s = 0; s < ns; s += 2) {
        meas_elem.push_back(i);
        meas_sp.push_back(s);
        tau.push_back(i % 3 == 0 ? 0.5 : 1.0);
        y.push_back(0.3);
        sigma.push_back(0.05);
      }
    lo.assign(np, -5.0);
    hi.assign(np, 5.0);
    refresh();
  }
  void add(int a, int b, int c, int e) {
    react.push_back(a);
    react.push_back(b);
    prod.push_back(c);
    prod.push_back(e);
    param.push_back(0);
    logk.push_back(-1.0);
  }
  void refresh() {
    d.n_s = ns;
    d.n_r = nr;
    d.n_p = np;
    d.N = N;
    d.react = react.data();
    d.prod = prod.data();
    d.param = param.data();
    d.logk_fixed = logk.data();
    d.h = h.data();
    d.z0 = z0.data();
    d.n_meas = (int)meas_elem.size();
    d.meas_elem = meas_elem.data();
    d.meas_species = meas_sp.data();
    d.meas_tau = tau.data();
    d.meas_y = y.data();
    d.meas_sigma = sigma.data();
    d.theta_lo = lo.data();
    d.theta_hi = hi.data();
  }
};

static void expect_valid(const colloc_instance_desc* d, int n, int K) {
  colloc_problem* p = nullptr;
  const int rc = colloc_create(d, n, K, &p);
  EXPECT(rc == COLLOC_OK);
  if (rc != COLLOC_OK) return;
  colloc_layout lay;
  EXPECT(colloc_layout_get(p, &lay) == COLLOC_OK);
  EXPECT(lay.n_inst == n && lay.K == K);
  EXPECT(colloc_table_bytes(p) > 0);
  EXPECT(colloc_workspace_bytes(p, COLLOC_FP64) > 0);
  EXPECT(colloc_workspace_bytes(p, COLLOC_FP32_IR) == colloc_workspace_bytes(p, COLLOC_FP64));
  EXPECT(colloc_workspace_bytes(p, 7) == 0);
  EXPECT(colloc_state_bytes(p) > 0);
  colloc_state_layout sl;
  EXPECT(colloc_state_layout_get(p, &sl) == COLLOC_OK);
  EXPECT(colloc_destroy(p) == COLLOC_OK);
}

static void expect_invalid(const colloc_instance_desc* d, int n, int K) {
  colloc_problem* p = (colloc_problem*)0x1;
  const int rc = colloc_create(d, n, K, &p);
  EXPECT(rc == COLLOC_EINVAL);
}

int main() {
  Net a(6, 7), b(6, 11);
  // valid: register path at every order, a batch of uneven meshes, then the tiled path
  for (int K = 1; K <= 5; ++K) expect_valid(&a.d, 1, K);
  colloc_instance_desc two[2] = {a.d, b.d};
  expect_valid(two, 2, 3);
  setenv("COLLOC_FACTOR_PATH", "tiled", 1);
  for (int K = 1; K <= 5; ++K) expect_valid(two, 2, K);
  unsetenv("COLLOC_FACTOR_PATH");
  // invalid: arguments, orders, shapes, indices and values
  colloc_problem* p = nullptr;
  EXPECT(colloc_create(nullptr, 1, 3, &p) == COLLOC_EINVAL);
  EXPECT(colloc_create(&a.d, 1, 3, nullptr) == COLLOC_EINVAL);
  expect_invalid(&a.d, 0, 3);
  expect_invalid(&a.d, 1, 0);
  expect_invalid(&a.d, 1, 6);
  Net c = a;
  c.refresh();
  c.d.N = 0;
  expect_invalid(&c.d, 1, 3);
  c.refresh();
  c.react[3] = c.ns;   // species index out of range
  expect_invalid(&c.d, 1, 3);
  c = a;
  c.refresh();
  c.param[0] = c.np;   // parameter index out of range
  expect_invalid(&c.d, 1, 3);
  c = a;
  c.refresh();
  c.h[2] = 0.0;        // element width not positive
  expect_invalid(&c.d, 1, 3);
  c = a;
  c.refresh();
  c.meas_elem[0] = c.N;   // measurement outside the mesh
  expect_invalid(&c.d, 1, 3);
  c = a;
  c.refresh();
  c.tau[1] = 1.5;      // local time outside [0, 1]
  expect_invalid(&c.d, 1, 3);
  c = a;
  c.refresh();
  c.sigma[0] = -1.0;   // noise scale not positive
  expect_invalid(&c.d, 1, 3);
  c = a;
  c.refresh();
  c.lo[0] = NAN;       // bounds not ordered
  expect_invalid(&c.d, 1, 3);
  c = a;
  c.refresh();
  c.z0[1] = INFINITY;  // initial state not finite
  expect_invalid(&c.d, 1, 3);
  Net e(5, 4);
  colloc_instance_desc mixed[2] = {a.d, e.d};
  expect_invalid(mixed, 2, 3);   // instances of different shape classes
  // host-side checks of the other entry points: null handles and pointers
  EXPECT(colloc_destroy(nullptr) == COLLOC_EINVAL);
  EXPECT(colloc_table_bytes(nullptr) == 0);
  EXPECT(colloc_state_bytes(nullptr) == 0);
  colloc_layout lay;
  EXPECT(colloc_layout_get(nullptr, &lay) == COLLOC_EINVAL);
  if (failures) {
    fprintf(stderr, "%d expectation(s) failed\n", failures);
    return 1;
  }
  printf("host validation: all expectations met\n");
  return 0;
}
