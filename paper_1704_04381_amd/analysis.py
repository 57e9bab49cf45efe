"""Scaling analysis of Rosenbluth ensembles (Sec. 4 of the paper).

Two fits over a series of chain lengths, both ordinary or weighted linear
least squares on logarithms:

* Eq. 4, <R_N^2> = a N^(2 nu): log <R^2> = log a + 2 nu log n.
* Eqs. 5 and 7, Z_N ~ mu^N N^(gamma - 1) with Z_N estimated by the mean
  Rosenbluth weight (Eq. 6): log Z = c + n log mu + (gamma - 1) log n.

Here n = N - 1 is the number of bonds (steps).  With m_1 counted in W the
mean weight estimates c_n, the number of n-step self-avoiding walks, so the
fit is the standard c_n ~ A mu^n n^(gamma - 1).  The paper writes both laws
with N; the exponents are the same for either choice, and only the
amplitudes and the corrections to scaling differ.

The sweep runs every chain length of the series as one batched GPU call
(``gen_batch``); the fits are host-side numpy.  Plain Rosenbluth weights
degenerate as N grows (the effective sample size, reported per row, falls
by orders of magnitude), so the weighted averages of long chains need many
more chains than short ones; fits should use lengths whose ESS is large.
"""
from __future__ import annotations

import math

import numpy as np


def _lstsq(X, y, sigma=None):
    """Least-squares solution, its covariance and the residual chi^2 per
    degree of freedom.  Without sigma the covariance is scaled by the
    residual variance (errors estimated from the scatter)."""
    X = np.asarray(X, dtype=np.float64)
    y = np.asarray(y, dtype=np.float64)
    if sigma is not None:
        w = 1.0 / np.asarray(sigma, dtype=np.float64)
        Xw, yw = X * w[:, None], y * w
    else:
        Xw, yw = X, y
    beta, *_ = np.linalg.lstsq(Xw, yw, rcond=None)
    r = yw - Xw @ beta
    dof = max(len(y) - X.shape[1], 1)
    chi2 = float(r @ r) / dof
    cov = np.linalg.pinv(Xw.T @ Xw)
    if sigma is None:
        cov = cov * chi2
    return beta, cov, chi2


def fit_nu(N, r2, r2_err=None):
    """nu and a of <R^2> = a n^(2 nu), n = N - 1, from mean squared
    end-to-end distances (optionally with their standard errors)."""
    n = np.asarray(N, dtype=np.float64) - 1.0
    r2 = np.asarray(r2, dtype=np.float64)
    X = np.stack([np.ones_like(n), np.log(n)], axis=1)
    sig = None if r2_err is None else np.asarray(r2_err, dtype=np.float64) / r2
    beta, cov, chi2 = _lstsq(X, np.log(r2), sig)
    return dict(nu=beta[1] / 2.0, nu_err=math.sqrt(max(cov[1, 1], 0.0)) / 2.0,
                a=math.exp(beta[0]), chi2_dof=chi2)


def fit_mu_gamma(N, log_z, log_z_err=None):
    """mu, gamma and log A of log Z = log A + n log mu + (gamma - 1) log n,
    n = N - 1, from log mean Rosenbluth weights."""
    n = np.asarray(N, dtype=np.float64) - 1.0
    X = np.stack([np.ones_like(n), n, np.log(n)], axis=1)
    beta, cov, chi2 = _lstsq(X, log_z, log_z_err)
    mu = math.exp(beta[1])
    return dict(mu=mu, mu_err=mu * math.sqrt(max(cov[1, 1], 0.0)),
                gamma=beta[2] + 1.0, gamma_err=math.sqrt(max(cov[2, 2], 0.0)),
                log_a=beta[0], chi2_dof=chi2)


def scaling_sweep(geometry, Ns, n_chains, seed=1, k=None, bond_length=1.0, bead_diameter=1.0):
    """Grow one ensemble per chain length (all in one batched call) and fit.

    Returns a dict with the per-N summaries ("rows") and the fits "nu" and,
    on the lattice, "mu_gamma" (for hard spheres the mean weight is the
    free-volume product times k^n, whose growth rate is not a lattice
    connective constant; the fit is still returned).
    """
    from . import gen_batch

    if k is None:
        k = 6 if geometry == "lattice" else 8
    specs = []
    for i, N in enumerate(Ns):
        sp = dict(geometry=geometry, N=int(N), k=k, n_chains=int(n_chains), seed=int(seed) + i)
        if geometry == "real":
            sp.update(bond_length=bond_length, bead_diameter=bead_diameter)
        specs.append(sp)
    res = gen_batch(specs, per_chain=False)
    rows = []
    for N, (_, s) in zip(Ns, res):
        rows.append(dict(N=int(N), n_alive=s["n_alive"], log_c_est=s["log_c_est"],
                         c_rel_err=s["c_rel_err"], r2_mean=s["r2_mean"], r2_err=s["r2_err"],
                         rg2_mean=s["rg2_mean"], rg2_err=s["rg2_err"], ess=s["ess"]))
    Nv = [r["N"] for r in rows]
    nu = fit_nu(Nv, [r["r2_mean"] for r in rows], [r["r2_err"] for r in rows])
    mg = fit_mu_gamma(Nv, [r["log_c_est"] for r in rows], [r["c_rel_err"] for r in rows])
    return dict(rows=rows, nu=nu, mu_gamma=mg)
