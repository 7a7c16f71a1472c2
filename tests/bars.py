"""Error bars of the GPU parity tests, scaled to the size of what is compared.

Amplitudes of an n-qubit state are about 2^(-n/2) in size, so an absolute
bar says little at large n.  Each check here measures the error against the
scale of the compared quantity and prints it, so a run's log records the
margin as well as the verdict.
"""
import numpy as np

EPS = {"c64": 2.0 ** -24, "c128": 2.0 ** -53}   # unit roundoff of the run's real type


def amp_error(got, ref):
    """max_j |got_j - ref_j| / max_j |ref_j|."""
    got, ref = np.asarray(got), np.asarray(ref)
    return float(np.max(np.abs(got - ref)) / max(np.max(np.abs(ref)), 1e-300))


def assert_amps(got, ref, dtype, ops, label=""):
    """A unitary evolution of `ops` gate (or block) applications in the run's
    precision: each application moves an amplitude by a few roundoffs of the
    amplitudes it mixes, so the error stays below 8 * ops * eps times the
    state's largest amplitude (a worst-case linear growth; the observed growth
    is closer to sqrt(ops))."""
    err = amp_error(got, ref)
    bar = 8.0 * max(ops, 1) * EPS[dtype]
    print(f"amps {label} {dtype}: max|d|/max|ref| = {err:.2e} (bar {bar:.1e})", flush=True)
    assert err <= bar, (label, err, bar)


def assert_hpsi(got, ref, psi, coeffs, dtype, label=""):
    """(H psi)_j = sum_k c_k phase_k psi_(j xor x_k): a sum of T terms each at
    most |c_k| max|psi| in size, so the error stays below 4 T eps S max|psi|."""
    got, ref = np.asarray(got), np.asarray(ref)
    T = len(coeffs)
    scale = float(np.abs(coeffs).sum()) * float(np.max(np.abs(psi)))
    err = float(np.max(np.abs(got - ref))) / scale
    bar = 4.0 * T * EPS[dtype]
    print(f"H psi {label} {dtype}: max|d|/(S max|psi|) = {err:.2e} (bar {bar:.1e})", flush=True)
    assert err <= bar, (label, err, bar)


def assert_grad_components(got, ref, rtol, floor, label=""):
    """Per component: |g_i - r_i| <= rtol |r_i| + floor max|r|.  The floor
    covers components near zero, whose error is set by the overall gradient
    scale, not by their own size."""
    got, ref = np.asarray(got), np.asarray(ref)
    scale = float(np.max(np.abs(ref)))
    d = np.abs(got - ref)
    worst_rel = float(np.max(d / (np.abs(ref) + floor / rtol * scale)))
    print(f"grad {label}: max|d| = {float(d.max()):.2e}, max|r| = {scale:.2e}, "
          f"max |d|/(|r| + {floor / rtol:.0e} max|r|) = {worst_rel:.2e} (bar {rtol:.0e})", flush=True)
    assert np.all(d <= rtol * np.abs(ref) + floor * scale), (label, worst_rel)
