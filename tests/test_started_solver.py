"""Host logic of warmstart.StartedSolver (stall check, continuation, cold
restart), with the batch and single-slice solvers replaced by stand-ins that
replay given relative-update histories (no GPU)."""
import pytest

pytest.importorskip("torch")

TOL = 1e-4


class FakeGeom:
    def __init__(self, warm, cold):
        self.warm, self.cold = warm, cold   # relative update after each iteration, warm / cold start


class FakeBatch:
    """Batch stand-in: image = number of iterations taken from the start."""

    def __init__(self, geoms, *, init, max_outer, tol, **kw):
        assert init == "user"
        self.geoms, self.K, self.tol = geoms, max_outer, tol
        self.calls = []

    def solve(self, ys, ws, fs, active=None):
        n = len(self.geoms)
        active = [True] * n if active is None else list(active)
        self.calls.append(active)
        its, rels, sts = [0] * n, [0.0] * n, [0] * n
        fs = list(fs)
        for j, g in enumerate(self.geoms):
            if not active[j]:
                continue
            k0 = fs[j]
            k = 0
            while k < self.K:
                k += 1
                r = g.warm[min(k0 + k, len(g.warm)) - 1]
                if r < self.tol:
                    break
            fs[j], its[j], rels[j] = k0 + k, k, r
            sts[j] = 0 if r < self.tol else 1
        return fs, its, rels, sts, max(sts)

    def close(self):
        pass


class FakeRecon:
    def __init__(self, g, max_outer, tol):
        self.g, self.K, self.tol = g, max_outer, tol
        self.used = False

    @classmethod
    def from_geometry(cls, g, *, max_outer, tol, **kw):
        return cls(g, max_outer, tol)

    def solve(self, y, w):
        self.used = True
        for k in range(1, self.K + 1):
            r = self.g.cold[min(k, len(self.g.cold)) - 1]
            if r < self.tol:
                return "cold", k, r, 0
        return "cold", self.K, r, 1

    def close(self):
        pass


def geometric(r0, q, n):
    return [r0 * q ** k for k in range(n)]


@pytest.fixture
def solver(monkeypatch):
    import paper_1009_1351_amd.recon as recon_mod
    monkeypatch.setattr(recon_mod, "Batch", FakeBatch)
    monkeypatch.setattr(recon_mod, "Recon", FakeRecon)
    from paper_1009_1351_amd.warmstart import StartedSolver

    def make(geoms, **kw):
        return StartedSolver(geoms, patch=7, window=15, h=0.01, mu_hat=0.5, tol=TOL, max_outer=600,
                             restart_after=64, **kw)
    return make


def test_stall_check_restarts_cycling_slices_early(solver):
    fast = FakeGeom(geometric(1e-2, 0.5, 100), [])                 # below 1e-4 after 8 iterations
    slow = FakeGeom(geometric(1e-2, 0.92, 200), [])                # 0.92^10 = 0.43 per 10: continues, converges at 57
    cyc = FakeGeom([3e-3 if k % 2 else 2.9e-3 for k in range(700)], geometric(1e-2, 0.9, 200))
    late = FakeGeom(geometric(1e-2, 0.95, 400), geometric(1e-2, 0.8, 100))   # 0.95^10 = 0.599: passes the check
    sol = solver([fast, slow, cyc, late])
    fs, its, st = sol.solve([None] * 4, [None] * 4, [0] * 4)
    assert its[0] == 8 and st[0] == 0 and fs[0] == 8
    assert its[1] == 57 and st[1] == 0
    # the cycling slice leaves after 20 warm iterations and converges cold
    cold_its = next(k for k in range(1, 200) if 1e-2 * 0.9 ** (k - 1) < TOL)
    assert its[2] == 20 + cold_its and st[2] == 0 and fs[2] == "cold"
    # the slowly converging one passes the check, is not done after 64, restarts then
    late_cold = next(k for k in range(1, 100) if 1e-2 * 0.8 ** (k - 1) < TOL)
    assert its[3] == 64 + late_cold and st[3] == 0 and fs[3] == "cold"
    # second segment only for the slices still running after the first; the
    # rest of the batch only for the ones that passed the check
    assert sol.seg.calls == [[True] * 4, [False, True, True, True]]
    assert sol.rest.calls == [[False, True, False, True]]


def test_without_stall_check_only_the_late_restart(solver):
    cyc = FakeGeom([3e-3] * 700, geometric(1e-2, 0.9, 200))
    sol = solver([cyc], stall_window=None)
    fs, its, st = sol.solve([None], [None], [0])
    cold_its = next(k for k in range(1, 200) if 1e-2 * 0.9 ** (k - 1) < TOL)
    assert sol.seg is None and its[0] == 64 + cold_its and fs[0] == "cold"
