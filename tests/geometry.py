"""Small seeded test geometries (inputs only)."""
import numpy as np

from paper_2504_19941_amd import workloads as W


def wall_and_particle(dim, shape, thickness=4, radius=5.0, seed=0):
    """Flat bottom wall plus a solid disc / ball above it: C1 is the tanh of
    the larger of the two signed distances, so the surface has curved and flat
    parts and cut links with q spread over (0, 1)."""
    rng = np.random.default_rng(seed)
    X = np.meshgrid(*[np.arange(n, dtype=np.float64) for n in shape], indexing="ij")
    ax = dim - 1
    d_wall = W.periodic_slab_distance(X[ax], -0.5, thickness - 0.5, shape[ax])
    centre = [0.3 * n + rng.uniform(0, 1) for n in shape]
    centre[ax] = thickness + radius + 2.3
    r2 = sum(W.min_image(X[d] - centre[d], shape[d]) ** 2 for d in range(dim))
    d_ball = radius - np.sqrt(r2)
    C1 = W.tanh_profile(np.maximum(d_wall, d_ball))
    mask = (np.maximum(d_wall, d_ball) > 0).astype(np.uint8)
    drop_c = [0.7 * n for n in shape]
    drop_c[ax] = thickness - 0.5
    C2 = W.drop_field(shape, drop_c, 0.3 * min(shape), C1, open_axis=ax)
    return mask, C1, C2
