"""Comparison helpers for the GPU-vs-oracle parity tests (no method arithmetic)."""
import numpy as np


def probe_errors(got: dict, ref: dict):
    """Per-probe error under the waveform rule: relative L2 ||g - o|| / ||o||,
    except that a probe whose ||o|| is below 1e-3 of the largest probe norm
    is measured against that largest norm (its relative error is
    ill-conditioned)."""
    norms = {k: float(np.linalg.norm(ref[k])) for k in ref}
    big = max(norms.values())
    out = {}
    for k in ref:
        g, o = np.asarray(got[k]), np.asarray(ref[k])
        assert g.shape == o.shape, (k, g.shape, o.shape)
        d = float(np.linalg.norm(g - o))
        den = norms[k] if norms[k] >= 1e-3 * big else big
        out[k] = d / den if den > 0 else d
    return out


def assert_probes_close(got: dict, ref: dict, tol: float):
    errs = probe_errors(got, ref)
    worst = max(errs, key=errs.get)
    assert errs[worst] <= tol, f"worst probe {worst}: {errs[worst]:.3e} > {tol:.1e}; all={errs}"
    return errs
