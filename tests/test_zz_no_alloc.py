"""The allocation-free A apply (wb_apply_A_noalloc) against wb_apply_A through the C-ABI: the
same operator and kernels with the library's fixed per-device workspace instead of an allocated
one.  Two calls in a row, the second on a smaller mesh (the workspace keeps the first call's
contents); a mesh whose workspace does not fit is rejected before any launch."""
import numpy as np
import pytest

from synthetic import WORKLOADS, custom, random_vector

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _wb():
    from paper_1607_03936_amd import wbfbt
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    wbfbt.lib()
    return wbfbt


def _apply_both(wb, w, seed):
    m = wb.Mesh(w.N, w.k)
    v = wb.Viscosity.sinker(m, w.centers(), w.delta, w.omega, w.mu_min, w.mu_max)
    u = torch.as_tensor(random_vector(seed, m.u_len), device="cuda")
    y_ref = torch.empty_like(u)
    y = torch.full_like(u, float("nan"))
    wb.wb_apply_A(m, v, u, y_ref)
    wb.wb_apply_A_noalloc(m, v, u, y)
    torch.cuda.synchronize()
    return y_ref.cpu().numpy(), y.cpu().numpy()


def test_noalloc_apply_matches_apply_twice():
    wb = _wb()
    # 48^3 Q2 (brick form: its two-pass buffer exceeds the fixed workspace), then a smaller
    # mesh in the two-pass form, then the 32^3 Q2 workload
    for w, seed in ((WORKLOADS["c4"], 61), (custom("n12k3", 12, 3, n_sinkers=5, dr=1e8, seed=62), 63),
                    (WORKLOADS["c2"], 64)):
        want, got = _apply_both(wb, w, seed)
        assert np.all(np.isfinite(got))
        assert np.abs(got - want).max() <= 1e-12 * np.abs(want).max(), w.name


def test_noalloc_rejects_a_mesh_whose_workspace_does_not_fit():
    wb = _wb()
    w = WORKLOADS["c5"]
    m = wb.Mesh(w.N, w.k)
    v = wb.Viscosity.sinker(m, w.centers(), w.delta, w.omega, w.mu_min, w.mu_max)
    u = torch.zeros(m.u_len, dtype=torch.float64, device="cuda")
    y = torch.zeros_like(u)
    with pytest.raises(wb.WbError) as ei:
        wb.wb_apply_A_noalloc(m, v, u, y)
    assert ei.value.code == wb.WB_EINVAL and "workspace" in str(ei.value)
