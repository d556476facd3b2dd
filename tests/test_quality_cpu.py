"""The sequential objective Phi_seq used for solution quality, pinned by the closed-form solution
of the linear A <-> B system: A(t) = A_inf + (A0 - A_inf) exp(-(k1 + k2) t) with
A_inf = k2 (A0 + B0) / (k1 + k2), measured in [A]; and the measurement times of a mesh."""
import numpy as np

from paper_2607_12201_amd import quality, workloads


def _closed_form_phi(inst, theta):
    k1, k2 = np.exp(theta)
    a0, b0 = inst["z0"]
    ainf = k2 * (a0 + b0) / (k1 + k2)
    t = quality.measurement_times(inst)
    pred = ainf + (a0 - ainf) * np.exp(-(k1 + k2) * t)
    r = (inst["meas_y"] - pred) / inst["meas_sigma"]
    return 0.5 * float(r @ r)


def test_measurement_times_are_element_ends():
    inst = workloads.ab_reversible(0)
    t = quality.measurement_times(inst)
    ends = np.cumsum(inst["h"])
    assert np.allclose(t, ends[inst["meas_elem"]], rtol=0, atol=1e-13)


def test_sequential_objective_matches_closed_form():
    inst = workloads.ab_reversible(0)
    for theta in (inst["theta_true"], inst["theta0"], np.array([1.5, -2.0])):
        ref = _closed_form_phi(inst, theta)
        got = quality.sequential_objective(inst, theta)
        assert abs(got - ref) <= 1e-7 * max(1.0, ref), (got, ref)


def test_relative_objective_gap():
    inst = workloads.ab_reversible(0)
    th = inst["theta_true"]
    assert quality.relative_objective_gap(inst, th, th) == 0.0
    other = th + np.array([0.3, -0.2])
    g = quality.relative_objective_gap(inst, other, th)
    ref = abs(_closed_form_phi(inst, other) - _closed_form_phi(inst, th)) / _closed_form_phi(inst, th)
    assert abs(g - ref) <= 1e-6 * max(1.0, ref)


def test_refine_uniform_maps_measurements_and_interpolates_polynomials():
    """Halving the mesh keeps every measurement at its absolute time, and the warm start
    reproduces states that are polynomials of degree <= K in time exactly."""
    from paper_2607_12201_amd import colloc
    inst = workloads.ab_reversible(0)
    K = 3
    tau, _ = colloc.library_tables(K)
    N, ns = inst["N"], inst["n_s"]
    starts = np.concatenate([[0.0], np.cumsum(inst["h"])[:-1]])
    t_nodes = starts[:, None] + np.asarray(inst["h"])[:, None] * tau[None, :]
    poly = lambda t: np.stack([1 + 0.3 * t - 0.05 * t ** 2 + 0.002 * t ** 3, 2 - t ** 3 / 100], axis=-1)
    x = np.concatenate([poly(t_nodes).ravel(), inst["theta0"]])
    new, x0 = quality.refine_uniform(inst, K, x)
    assert new["N"] == 2 * N
    assert np.allclose(quality.measurement_times(new), quality.measurement_times(inst), rtol=0, atol=1e-12)
    starts2 = np.concatenate([[0.0], np.cumsum(new["h"])[:-1]])
    t2 = starts2[:, None] + np.asarray(new["h"])[:, None] * tau[None, :]
    assert np.allclose(x0[: 2 * N * (K + 1) * ns], poly(t2).ravel(), rtol=0, atol=1e-12)
    assert np.array_equal(x0[2 * N * (K + 1) * ns:], inst["theta0"])
