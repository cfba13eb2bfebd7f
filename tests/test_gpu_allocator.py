"""gl_set_allocator: the handles' device workspaces from PyTorch's caching
allocator (glnk.use_torch_allocator).  The memory shows up in torch's
accounting while the handles live and goes back when they are destroyed;
results are bitwise those of the hipMalloc path."""
import gc

import numpy as np
import pytest

from paper_1204_5125_amd import inputs

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def glnk():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1204_5125_amd import glnk as g
    g.lib()
    return g


def run(glnk, psi0):
    mesh = glnk.Mesh(2, (65, 65), (8.0, 8.0), mu=0.7)
    psi = torch.from_numpy(psi0).cuda()
    pre = glnk.PrecondHandle(mesh)
    rc, info = glnk.gl_newton_solve(mesh, psi, tol=1e-10, max_steps=30, precond=pre)
    torch.cuda.synchronize()
    return mesh, pre, rc, info, psi.cpu().numpy()


def test_torch_allocator_backs_the_workspaces(glnk):
    psi0 = inputs.random_phase_state(65 * 65, seed=81)
    m0, p0, rc0, i0, ref = run(glnk, psi0)
    p0.close()
    m0.close()
    gc.collect()
    torch.cuda.synchronize()
    base = torch.cuda.memory_allocated()
    glnk.use_torch_allocator()
    try:
        mesh, pre, rc, info, out = run(glnk, psi0)
        held = torch.cuda.memory_allocated() - base
        # the mesh alone holds 11 Krylov vectors of n complex doubles
        assert held >= 11 * 16 * 65 * 65
        assert rc == rc0 == 0 and info == i0
        assert np.array_equal(out, ref)
        pre.close()
        mesh.close()
        gc.collect()
        torch.cuda.synchronize()
        assert torch.cuda.memory_allocated() <= base
    finally:
        glnk.gl_set_allocator(None, None)
    # hipMalloc again
    m2, p2, rc2, i2, out2 = run(glnk, psi0)
    assert np.array_equal(out2, ref)
    # one function without the other is rejected
    rc = glnk.lib().gl_set_allocator(glnk._ALLOC_FN(lambda n, s, c: None), glnk._FREE_FN(), None)
    assert rc == 1
