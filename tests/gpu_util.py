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


def grid_grad_magnitude(grid, pos, scale, w):
    """Magnitude sum of the grid force at each point, per axis (n, 3):
    sum_c |w_c| |de_c/dv| (1/h) sum_q W_q |g_qc|, the trilinear gradient's
    corner terms taken in absolute value (W_q the corner's weight in the two
    other axes; de/dv = s for a plain channel, 4 s v^3 for a quartic-root
    one).  A float32 gradient differences corner values; deep in a capped
    region they are large and nearly equal, and its rounding scales with
    this sum rather than with the force itself."""
    pos = np.asarray(pos, np.float64)
    nodes = grid.nodes.astype(np.float64)
    n3 = np.array(grid.n)
    u = np.clip((pos - np.asarray(grid.origin)) / grid.spacing, -1, n3)
    i = np.clip(np.floor(u).astype(np.int64), 0, n3 - 2)
    t = np.clip(u - i, 0.0, 1.0)
    corners = {}
    for a in (0, 1):
        for b in (0, 1):
            for c in (0, 1):
                corners[a, b, c] = nodes[i[:, 2] + c, i[:, 1] + b, i[:, 0] + a]
    v = np.zeros((len(pos), nodes.shape[-1]))
    for (a, b, c), g in corners.items():
        v += ((t[:, 0] if a else 1 - t[:, 0]) * (t[:, 1] if b else 1 - t[:, 1])
              * (t[:, 2] if c else 1 - t[:, 2]))[:, None] * g
    quart = np.asarray(grid.transform) == 4
    s = np.abs(np.asarray(scale, np.float64))
    dedv = np.where(quart[None], 4.0 * s * np.abs(v) ** 3, s)
    out = np.zeros((len(pos), 3))
    for ax in range(3):
        acc = np.zeros_like(v)
        for bits, g in corners.items():
            wp = np.ones(len(pos))
            for o in range(3):
                if o != ax:
                    wp *= t[:, o] if bits[o] else 1 - t[:, o]
            acc += wp[:, None] * np.abs(g)
        out[:, ax] = (np.abs(np.asarray(w))[None] * dedv * acc).sum(1) / \
            grid.spacing
    return out
