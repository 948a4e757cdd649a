"""Host logic of the reverse sweep (paper_1601_07944_amd.adjoint), no GPU:
the checkpointed sweep and the keep-all tape chain the step adjoints over
the right states in the right order.  A stand-in mesh object maps a state
elementwise, C -> C + dt sin(C), with stage states u1 = sin(C), u2 = cos(C)
and the step adjoint g -> g (1 + dt cos(C)); the gradient of N such steps is
the product of the factors, which torch's autograd gives independently."""
import pytest
import torch

from paper_1601_07944_amd import adjoint as A


class StepStandIn:
    def __init__(self, n):
        self.n = n
        self.vjp_inputs = []

    def empty_state(self):
        return torch.empty(self.n, dtype=torch.float64)

    def rk_step(self, C, dt):
        C.add_(dt * torch.sin(C))

    def rk_step_stages_to(self, C, Cnext, u1, u2, dt):
        u1.copy_(torch.sin(C))
        u2.copy_(torch.cos(C))
        Cnext.copy_(C + dt * u1)

    def rk_step_vjp(self, C, g, dt, u1=None, u2=None):
        # the stage states must be those of this step's input
        assert torch.equal(u1, torch.sin(C)) and torch.equal(u2, torch.cos(C))
        self.vjp_inputs.append(C.clone())
        return g * (1.0 + dt * u2)


def reference(C0, dt, nsteps, gN):
    x = C0.clone().requires_grad_(True)
    C = x
    for _ in range(nsteps):
        C = C + dt * torch.sin(C)
    C.backward(gN)
    return C.detach(), x.grad


@pytest.mark.parametrize("every", [0, 1, 4, 7, 23, 40])
def test_sweep_gradient_and_order(every):
    n, nsteps, dt = 64, 23, 0.05
    g = torch.Generator().manual_seed(3)
    C0 = torch.randn(n, dtype=torch.float64, generator=g)
    gN = torch.randn(n, dtype=torch.float64, generator=g)
    CN_ref, g_ref = reference(C0, dt, nsteps, gN)
    dm = StepStandIn(n)
    x = C0.clone().requires_grad_(True)
    CN = A.run_steps(x, dm, dt, nsteps, every)
    CN.backward(gN)
    assert torch.allclose(CN.detach(), CN_ref, rtol=1e-14, atol=0)
    assert torch.allclose(x.grad, g_ref, rtol=1e-13, atol=0)
    # the adjoints ran last step first, over the states C_{N-1}, ..., C_0
    states = [C0.clone()]
    for _ in range(nsteps - 1):
        states.append(states[-1] + dt * torch.sin(states[-1]))
    assert len(dm.vjp_inputs) == nsteps
    for got, want in zip(dm.vjp_inputs, reversed(states)):
        assert torch.allclose(got, want, rtol=1e-14, atol=0)


def test_keep_all_tape_is_released_and_input_untouched():
    n, nsteps, dt = 16, 5, 0.1
    C0 = torch.linspace(-1, 1, n, dtype=torch.float64)
    keep = C0.clone()
    dm = StepStandIn(n)
    CN, tape = A.forward_keep_all(dm, C0.clone(), dt, nsteps)
    assert len(tape) == nsteps and torch.equal(tape[0][0], keep)
    A.backward_tape(dm, tape, dt, torch.ones(n, dtype=torch.float64))
    assert tape == []
    assert torch.equal(C0, keep)


def test_negative_interval_rejected():
    dm = StepStandIn(4)
    with pytest.raises(ValueError):
        A.run_steps(torch.zeros(4, dtype=torch.float64, requires_grad=True), dm, 0.1, 3, -1)
