"""A stepper over the CPU oracle (numpy arrays), for exercising the rollout
and checkpointing logic without a GPU and as the reference gradient."""
import oracle as O


class OracleStepper:
    def __init__(self, prob):
        self.p = O.Problem(prob)

    def copy(self, U):
        return U.copy()

    def step(self, U, dt=None):
        return O.step(self.p, U, dt)

    def step_vjp(self, Un, g, dt):
        return O.step_vjp(self.p, Un, dt, g)
