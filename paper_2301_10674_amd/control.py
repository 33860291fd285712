"""Flow-rate control of a flume.

Section 3.1 drives the flow by a body force F_x that is controlled during
the run to hold the bulk flow rate; the paper gives no control law.  The
law here (a reading) is proportional-integral on the bulk velocity: every
`every` steps, e = target - U_x (``fsl_bulk_velocity``), I += e and
a_x = a0 + kp e + ki I (``fsl_set_accel``).  This is host-side orchestration
of C-ABI calls; every step runs on the GPU.
"""


class FlowController:
    def __init__(self, target, a0, kp, ki, every):
        if every < 1:
            raise ValueError("every must be >= 1")
        self.target, self.a0, self.kp, self.ki, self.every = target, a0, kp, ki, every
        self.integral = 0.0
        self.accel = a0

    def run(self, lat, steps):
        """Advance `lat` by `steps` steps under control; returns the final a_x."""
        done = 0
        while done < steps:
            k = min(self.every, steps - done)
            lat.step(k)
            done += k
            err = self.target - float(lat.bulk_velocity()[0])
            self.integral += err
            self.accel = self.a0 + self.kp * err + self.ki * self.integral
            lat.set_accel((self.accel, 0.0, 0.0))
        return self.accel
