"""The truncation-error extrapolation (CPU only): the fit recovers known
polynomials exactly, estimates its own uncertainty from noisy points, and the
converged point of a long run is read from its last period records."""
import numpy as np

from paper_1606_06790_amd import extrapolate


def test_fit_recovers_a_quadratic():
    eps = np.array([8e-5, 6e-5, 4e-5, 2.5e-5, 1.5e-5, 9e-6])
    e = -0.43838 + 7.1 * eps - 2.0e3 * eps ** 2
    c, err0, rms = extrapolate.fit(eps, e, 2)
    assert abs(c[0] + 0.43838) <= 1e-12 and abs(c[1] - 7.1) <= 1e-6 and abs(c[2] + 2.0e3) <= 1e-2
    assert rms <= 1e-15 and err0 <= 1e-10


def test_fit_error_estimate_covers_noise():
    rng = np.random.default_rng(7)
    eps = np.linspace(1e-5, 1e-4, 8)
    hits = 0
    for _ in range(200):
        e = -0.4 + 5.0 * eps + rng.normal(0.0, 1e-7, eps.size)
        c, err0, _ = extrapolate.fit(eps, e, 1)
        hits += abs(c[0] + 0.4) <= 2 * err0
    assert hits >= 170          # about 95 % within two standard errors


def test_converged_point_reads_the_last_periods():
    recs = [dict(kind="config", m=800)] + [dict(kind="period", n=12 * k + 11, e_g=-0.4 - 1e-3 / (k + 1), eps=1e-5 * k)
                                           for k in range(6)]
    m, e, eps, spread = extrapolate.converged_point(recs, periods=3)
    assert m == 800 and e == recs[-1]["e_g"] and eps == recs[-1]["eps"]
    assert abs(spread - (recs[-1]["e_g"] - recs[-3]["e_g"])) <= 1e-15


def test_main_leaves_out_runs_below_m_min(tmp_path, capsys):
    paths = []
    for m, e, eps in ((400, -0.4352, 2.2e-4), (800, -0.43780, 8.7e-5), (1600, -0.43817, 3.1e-5),
                      (2800, -0.43829, 1.3e-5)):
        p = tmp_path / f"m{m}.jsonl"
        p.write_text("\n".join([f'{{"kind": "config", "m": {m}}}',
                                f'{{"kind": "period", "n": 11, "e_g": {e}, "eps": {eps}}}']) + "\n")
        paths.append(str(p))
    out = extrapolate.main(paths, m_min=600)
    text = capsys.readouterr().out
    assert "m=  400" in text and "left out" in text
    assert np.isnan(out[2]["e0_stderr"])          # three points: the quadratic fits exactly, no error estimate
    c, _, _ = extrapolate.fit([8.7e-5, 3.1e-5, 1.3e-5], [-0.43780, -0.43817, -0.43829], 1)
    assert abs(out[1]["e0"] - c[0]) <= 1e-15


def test_observables_fit_recovers_known_limits(tmp_path, capsys):
    """Synthetic observables runs whose class averages, spreads and correlation points are exact quadratics in eps:
    the fits return the eps -> 0 values, and the correlation length of an exact exponential."""
    import json
    xi = 0.7
    lines = []
    for m, eps in ((1200, 4.8e-5), (1600, 3.1e-5), (2000, 2.2e-5), (2400, 1.7e-5), (2800, 1.3e-5), (800, 8.7e-5)):
        cls = {"1-2": dict(average=-0.2158 + 3.0 * eps + 1e3 * eps ** 2, delta_plus=40.0 * eps,
                           delta_minus=-35.0 * eps - 2e4 * eps ** 2),
               "3-13": dict(average=-0.2208 - 2.0 * eps, delta_plus=eps, delta_minus=-eps)}
        vals = [(-1) ** r * 0.05 * np.exp(-r / xi) * (1 + 50 * eps) for r in range(1, 7)]
        lines.append(json.dumps(dict(m=m, n=239, eps=eps, classes=cls,
                                     correlation=dict(label=2, values=vals, xi_cells=xi))))
    p = tmp_path / "obs.jsonl"
    p.write_text("\n".join(lines) + "\n")
    out = extrapolate.observables([str(p)], eps_max=6e-5)
    assert len(out["points"]) == 5 and "left out" in capsys.readouterr().out
    assert abs(out["classes"]["1-2"]["average"]["value"] + 0.2158) <= 1e-12
    assert abs(out["classes"]["3-13"]["average"]["value"] + 0.2208) <= 1e-12
    assert abs(out["classes"]["1-2"]["delta_plus"]["value"]) <= 1e-12
    assert abs(out["classes"]["1-2"]["delta_minus"]["value"]) <= 1e-12
    assert abs(out["correlation"]["xi_cells"] - xi) <= 1e-9
    assert abs(out["correlation"]["values"][0] + 0.05 * np.exp(-1 / xi)) <= 1e-12
