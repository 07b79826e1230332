"""The deterministic assembly (fpde_params.deterministic = 1): the sums that
build K run in one wavefront per work item, so K is the same bit for bit on
every run, in FP64 and for the FP32 matrix of the mixed arm; and it equals
the default (fastest-order) assembly to rounding.  Between the two
deterministic assemblies another order alpha is assembled, so that the second
one recomputes every path value, merged entry and tube block."""
import pytest
import torch

import paper_1811_03339_amd as F
from fpde_inputs import workload_mesh

pytestmark = pytest.mark.gpu

_MESHES = {}


def gpu_mesh(name):
    if name not in _MESHES:
        m = workload_mesh(name)
        _MESHES[name] = F.Mesh(m.xyz, m.tet)
    return _MESHES[name]


@pytest.mark.parametrize("name,nq", [("sphere_small", 4), ("sphere20k", 11)])
@pytest.mark.parametrize("precision", [F.FPDE_FP64, F.FPDE_MIXED])
def test_deterministic_assembly_is_bit_stable(name, nq, precision):
    gm = gpu_mesh(name)
    n = gm.n_dof
    print(f"[deterministic] {name} n={n} nq={nq} precision={precision}", flush=True)
    dt = torch.float64 if precision == F.FPDE_FP64 else torch.float32
    A1 = torch.empty((n, n), dtype=dt, device="cuda")
    A2 = torch.empty_like(A1)
    A0 = torch.empty_like(A1)
    b = torch.empty(n, dtype=torch.float64, device="cuda")
    K = (1.0, 0.5, 2.0)
    p = F.params(1.5, K, quad_points=nq, precision=precision, deterministic=True)
    other = F.params(1.51, K, quad_points=nq, precision=precision, deterministic=True)
    gm.assemble(p, A1, b)
    gm.assemble(other, A0, b)
    gm.assemble(p, A2, b)
    torch.cuda.synchronize()
    assert torch.equal(A1, A2)
    gm.assemble(F.params(1.5, K, quad_points=nq, precision=precision), A0, b)
    torch.cuda.synchronize()
    rel = float((A0.double() - A1.double()).abs().max() / A1.double().abs().max())
    # FP64: the two summation orders of the same terms; FP32: at most the
    # rounding of the FP32 store differs
    assert rel <= (1e-13 if precision == F.FPDE_FP64 else 2e-7), rel
