"""One grid split into slabs along its last axis (z in 3D, y on D2Q9).

Each slab is a context whose cut faces use the LBM_HALO rule: its sweep
reads the populations entering through a cut from a receive buffer and packs
those leaving into a send buffer, and between steps each send buffer is moved
to the neighbour's receive buffer.  On several GPUs each slab would live on
its own device and the move would be a grouped send/recv; here all slabs share
one device and stream and `lbm_halo_exchange` does the move with device
copies.  The stepping is that of the undivided grid (the streaming of eq.
optimizedLB reads the same post-collision values), so results are bitwise
those of one context on the same sweep path.

Cells are numbered as in the undivided grid, c = (z*ny + y)*nx + x, so slab
k holds the contiguous cell range of its planes.  Inlet noise is drawn from
each slab's own cell numbering and therefore differs from the undivided run.
"""
from . import lbm


def split(n, k):
    """Plane counts of k slabs over n planes (the first n % k one larger)."""
    if not 1 <= k <= n:
        raise ValueError("cannot split %d planes into %d slabs" % (n, k))
    return [n // k + (1 if i < n % k else 0) for i in range(k)]


class Slabs:
    """k subdomains of one grid, stepped in lockstep with halo exchanges.

    Keyword arguments are those of `lbm.make_config` for the undivided grid;
    its last-axis faces decide the outer faces of the end slabs (both
    periodic: the slabs form a ring).
    """

    def __init__(self, k, shape, lattice=lbm.LBM_D3Q19, face_bc=(lbm.LBM_PERIODIC,) * 6,
                 sponge_width=(0,) * 6, **kw):
        import torch
        self.torch = torch
        d3 = lattice != lbm.LBM_D2Q9
        shape = (tuple(shape) + (1,))[:3]
        self.shape = shape
        ax = 2 if d3 else 1
        lo, hi = 2 * ax, 2 * ax + 1
        if sponge_width[lo] or sponge_width[hi]:
            raise ValueError("no face absorbing layer along the cut axis (use a per-cell layer)")
        self.ring = face_bc[lo] == lbm.LBM_PERIODIC
        # the undivided grid runs the periodic sweep path only when every face
        # is periodic, there is no layer and no mask; otherwise each slab is
        # given a mask (all FLUID if none) so that it runs the general path too
        self.general = (any(f != lbm.LBM_PERIODIC for f in face_bc)
                        or kw.get("chi_max", 0.0) > 0)
        self.sizes = split(shape[ax], k)
        self.plane = shape[0] * (shape[1] if d3 else 1)
        kw.setdefault("stream", torch.cuda.current_stream().cuda_stream)
        self.sims = []
        for i, n in enumerate(self.sizes):
            f = list(face_bc)
            f[lo] = lbm.LBM_HALO if (i > 0 or self.ring) else face_bc[lo]
            f[hi] = lbm.LBM_HALO if (i < k - 1 or self.ring) else face_bc[hi]
            s = list(shape)
            s[ax] = n
            self.sims.append(lbm.Simulation(lattice=lattice, shape=tuple(s), face_bc=tuple(f),
                                            sponge_width=tuple(sponge_width), **kw))
        self.q = lattice
        self.ranges = []
        c = 0
        for n in self.sizes:
            self.ranges.append((c, c + n * self.plane))
            c += n * self.plane
        self.ncell = c

    def exchange(self):
        lbm.lbm_halo_exchange([s.ctx for s in self.sims], self.ring)

    def init(self, rho=None, u=None, pi_neq=None, mask=None):
        """Fields of the undivided grid (host or device, layouts of lbm_init)."""
        t = self.torch
        dev = self.sims[0].device

        def dev_(a, dtype):
            if a is None:
                return None
            if not isinstance(a, t.Tensor):
                a = t.from_numpy(a)
            return a.to(device=dev, dtype=dtype)

        rho, u, pi_neq = dev_(rho, t.float64), dev_(u, t.float64), dev_(pi_neq, t.float64)
        mask = dev_(mask, t.uint8)
        if mask is None and self.general:
            mask = t.zeros(self.ncell, dtype=t.uint8, device=dev)
        if u is not None:
            u = u.reshape(-1, self.ncell)
        if pi_neq is not None:
            pi_neq = pi_neq.reshape(-1, self.ncell)
        for s, (c0, c1) in zip(self.sims, self.ranges):
            s.init(None if rho is None else rho[c0:c1].contiguous(),
                   None if u is None else u[:, c0:c1].contiguous(),
                   None if pi_neq is None else pi_neq[:, c0:c1].contiguous(),
                   None if mask is None else mask[c0:c1].contiguous())
        self.exchange()
        return self

    def step(self, n=1):
        for _ in range(n):
            for s in self.sims:
                s.step(1)
            self.exchange()
        return self

    def sync(self):
        for s in self.sims:
            s.sync()

    def moments(self):
        t = self.torch
        parts = [s.moments() for s in self.sims]
        return t.cat([p[0] for p in parts]), t.cat([p[1] for p in parts], dim=1)

    def populations(self):
        return self.torch.cat([s.populations() for s in self.sims], dim=1)

    def set_populations(self, f):
        for s, (c0, c1) in zip(self.sims, self.ranges):
            s.set_populations(f[:, c0:c1].contiguous())
        self.exchange()

    def close(self):
        for s in self.sims:
            s.close()
