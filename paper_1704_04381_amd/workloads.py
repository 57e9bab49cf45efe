"""Synthetic workloads of the Rosenbluth chain-growth path.

Definitions only: sizes and seeds, no arithmetic of the method.  Both the GPU
path and the oracle take a workload's (geometry, N, k, M, seed, ...) as input;
the random numbers are drawn inside the method from the counter-based stream.
The paper measures on chains it generates itself (10^6 chains per N, Tables 1
and 2); these are the configurations quoted for MI355X.
"""

WORKLOADS = {
    # Simple cubic lattice, N = 16 monomers, 10^5 chains, int32 coordinates,
    # exact integer weights W = prod m_i.
    "lattice_n16": dict(geometry="lattice", N=16, k=6, n_chains=100_000, seed=1,
                        coord="i32", exact_w=True, hist_bins=0),
    # Simple cubic lattice, N = 64, 10^7 chains, int16 coordinates, FP64 log W,
    # 256-bin W-weighted R^2 histogram.
    "lattice_n64": dict(geometry="lattice", N=64, k=6, n_chains=10_000_000, seed=1,
                        coord="i16", exact_w=False, hist_bins=256),
    # Hard-sphere chain in continuous space, b = sigma = 1, N = 64, k = 8 trial
    # directions, 10^6 chains, FP64.
    "real_n64": dict(geometry="real", N=64, k=8, n_chains=1_000_000, seed=1,
                     coord="f64", bond_length=1.0, bead_diameter=1.0, hist_bins=256),
    # 26-neighbour lattice variant (Sec. 3.3.2), N = 64, 10^7 chains, int16
    # coordinates, FP64 log W, 256-bin histogram.
    "lattice26_n64": dict(geometry="lattice26", N=64, k=26, n_chains=10_000_000, seed=1,
                          coord="i16", exact_w=False, hist_bins=256),
    # Long chains (LDS-resident group kernels): simple cubic lattice at
    # N = 256 (10^6 chains) and N = 2048 (10^5 chains), 26-neighbour lattice
    # likewise, int16 coordinates, FP64 log W, no histogram.
    "lattice_n256": dict(geometry="lattice", N=256, k=6, n_chains=1_000_000, seed=1,
                         coord="i16", exact_w=False, hist_bins=0),
    "lattice_n2048": dict(geometry="lattice", N=2048, k=6, n_chains=100_000, seed=1,
                          coord="i16", exact_w=False, hist_bins=0),
    "lattice26_n256": dict(geometry="lattice26", N=256, k=26, n_chains=1_000_000, seed=1,
                           coord="i16", exact_w=False, hist_bins=0),
    "lattice26_n2048": dict(geometry="lattice26", N=2048, k=26, n_chains=100_000, seed=1,
                            coord="i16", exact_w=False, hist_bins=0),
    # Long hard-sphere chains, k = 8, b = sigma = 1: N = 256 (bead planes in
    # LDS, 32 lanes per chain; 2 10^5 chains) and N = 3000 (bead planes in
    # HBM, one chain per wave of the persistent grid; 3 10^3 chains).
    "real_n256": dict(geometry="real", N=256, k=8, n_chains=200_000, seed=1,
                      coord="f64", bond_length=1.0, bead_diameter=1.0, hist_bins=0),
    "real_n3000": dict(geometry="real", N=3000, k=8, n_chains=3_000, seed=1,
                       coord="f64", bond_length=1.0, bead_diameter=1.0, hist_bins=0),
}


def steps_per_chain(w) -> int:
    """Nominal monomer-steps per chain (N - 1 growth steps)."""
    return w["N"] - 1


def mixed_ensembles(n=256, meta_seed=42, m_lo=3.0, m_span=3.0):
    """Descriptors of a mixed batch of ensembles (the batched-launch workload).

    Ensemble e draws three uniforms (u_N, u_k, u_M) from NumPy's
    Philox4x32-10 generator keyed by ``meta_seed`` (a published counter-based
    generator, so the list does not depend on the language that reads it):
    N = 8 + floor(121 u_N); even e are lattice ensembles (k = 6, int32 ends),
    odd e hard-sphere ensembles with k = 8 (u_k < 1/2) or 16 (b = sigma = 1);
    M = floor(10^(m_lo + m_span u_M)) chains; seed = meta_seed * 2^20 + e.
    Returns a list of dicts accepted by ``gen_chains`` / ``gen_batch``.
    """
    import numpy as np

    g = np.random.Generator(np.random.Philox(key=meta_seed))
    u = g.random((n, 3))
    out = []
    for e in range(n):
        N = 8 + int(121 * u[e, 0])
        M = int(10.0 ** (m_lo + m_span * u[e, 2]))
        seed = meta_seed * (1 << 20) + e
        if e % 2 == 0:
            out.append(dict(geometry="lattice", N=N, k=6, n_chains=M, seed=seed, coord="i32"))
        else:
            k = 8 if u[e, 1] < 0.5 else 16
            out.append(dict(geometry="real", N=N, k=k, n_chains=M, seed=seed, coord="f64",
                            bond_length=1.0, bead_diameter=1.0))
    return out


def serving_requests(n=2100, rate=200.0, meta_seed=7, m_lo=4.0, m_span=3.0):
    """Request stream of the serving workload: Poisson arrivals at ``rate``
    per second (exponential gaps) and per-request descriptors, all from
    NumPy's Philox4x32-10 keyed by ``meta_seed``.

    Request r draws (u_gap, u_N, u_geo, u_M): gap = -ln(1 - u_gap) / rate;
    N = (16, 32, 64, 128, 256)[floor(5 u_N)]; lattice (k = 6) when
    u_geo < 1/2, else hard spheres (k = 8, b = sigma = 1); M =
    floor(10^(m_lo + m_span u_M)) chains; seed = meta_seed * 2^20 + r.
    Returns a list of (arrival_seconds, spec) with spec as for ``gen_chains``.
    """
    import math

    import numpy as np

    g = np.random.Generator(np.random.Philox(key=meta_seed))
    u = g.random((n, 4))
    t = 0.0
    out = []
    for r in range(n):
        t += -math.log(1.0 - u[r, 0]) / rate
        N = (16, 32, 64, 128, 256)[min(int(5 * u[r, 1]), 4)]
        M = int(10.0 ** (m_lo + m_span * u[r, 3]))
        seed = meta_seed * (1 << 20) + r
        if u[r, 2] < 0.5:
            spec = dict(geometry="lattice", N=N, k=6, n_chains=M, seed=seed, coord="i32")
        else:
            spec = dict(geometry="real", N=N, k=8, n_chains=M, seed=seed, coord="f64",
                        bond_length=1.0, bead_diameter=1.0)
        out.append((t, spec))
    return out
