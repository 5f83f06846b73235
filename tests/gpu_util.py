"""Shared helpers of the GPU parity tests (not collected by pytest)."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")


def require_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU in this container")


def make_context(grid, ligs, seed, capacity=0):
    """Context with `grid` uploaded and every ligand of `ligs` set up."""
    import paper_1507_03703_amd as pkg
    ctx = pkg.Context(seed=seed, device=0)
    ctx.grid_upload(grid.nodes, grid.origin, grid.spacing, grid.transform)
    ids = [ctx.ligand_setup(l, sample_capacity=capacity) for l in ligs]
    return ctx, ids


def dev(a, dtype):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=dtype,
                           device="cuda:0").contiguous()


def near_face(pos, grid, extra=1e-6):
    """True where a coordinate lies within float32 rounding of a cell face
    (in cell units: within 4 ulp of the float32 grid coordinate), where the
    float32 and float64 paths may pick different cells and the one-sided
    trilinear gradient may legitimately differ."""
    pos = np.asarray(pos, np.float64)
    o = np.asarray(grid.origin, np.float64)
    u = (pos - o) / grid.spacing
    t = u - np.floor(u)
    d = np.minimum(t, 1.0 - t)
    ulp = np.spacing(np.abs(u).astype(np.float32)).astype(np.float64) + \
        np.spacing(np.abs(pos).astype(np.float32)).astype(np.float64) / \
        grid.spacing
    return np.any(d < 4 * ulp + extra, axis=-1)


def print_case(*args):
    print("CASE", *args, flush=True)
