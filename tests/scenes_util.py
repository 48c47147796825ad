"""Test helpers: convert scene descriptions into oracle inputs (no method arithmetic)."""
import oracle as O


def oracle_grid(sc):
    return O.Grid(sc.n, sc.n, sc.n, sc.dx)


def oracle_regions(sc):
    return [O.Region(kind=r.kind, lo=r.lo, hi=r.hi, center=r.center, radius=r.radius, vel=r.vel)
            for r in sc.regions]


def oracle_params(sc, tol=None, precond=O.PRECOND_MIC0, **kw):
    return O.Params(grid=oracle_grid(sc), gravity=sc.gravity, dt=sc.dt, flip_ratio=sc.flip_ratio,
                    density=sc.density, tol=sc.tol if tol is None else tol, precond=precond, **kw)
