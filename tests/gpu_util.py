"""Helpers shared by the GPU tests: device transfer and per-field errors."""
import numpy as np


def dev(a, dtype="f64"):
    import torch
    t = torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64))
    if dtype == "f32":
        t = t.float()
    return t.cuda()


def host(t):
    return t.detach().double().cpu().numpy()


def field_errors(x, ref):
    """Relative 2-norm error per field (and the max-norm analogue)."""
    out = []
    for k in range(ref.shape[0]):
        d = np.linalg.norm((x[k] - ref[k]).ravel())
        r = np.linalg.norm(ref[k].ravel())
        dm = np.abs(x[k] - ref[k]).max()
        rm = np.abs(ref[k]).max()
        out.append((d / max(r, 1e-300), dm / max(rm, 1e-300), r))
    return out


# per-field errors of every parity check of the session (printed as a table at
# the end of the run by conftest.py)
RECORDS = []


def assert_fields_close(x, ref, tol, what="", abs_floor=0.0):
    errs = field_errors(x, ref)
    RECORDS.append((what, tol, [e2 for e2, _, _ in errs], [em for _, em, _ in errs]))
    for k, (e2, em, r) in enumerate(errs):
        if r <= abs_floor:
            assert np.abs(x[k] - ref[k]).max() <= max(abs_floor, 1e-300), (what, k, "abs", np.abs(x[k] - ref[k]).max())
            continue
        assert e2 <= tol, f"{what}: field {k} rel-2 error {e2:.3e} > {tol:.1e} (max-norm {em:.3e})"
    return errs
