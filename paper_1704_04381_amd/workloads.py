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
}


def steps_per_chain(w) -> int:
    """Nominal monomer-steps per chain (N - 1 growth steps)."""
    return w["N"] - 1
