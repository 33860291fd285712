"""Four-way coupled time stepping of fluid and particles (Section 2.2).

One coupled step, in the order the coupling needs its data:

1. the fluid takes one lattice step with the spheres' current positions and
   velocities as moving walls (``Lattice.step``);
2. the hydrodynamic force and torque on every sphere follow by momentum
   exchange from the new state (``Lattice.particle_forces``);
3. the particles advance one lattice step of time in sub-steps under that
   load, gravity, collisions and lubrication (``Dem.step``);
4. the spheres are remapped onto the lattice at their new positions with
   their new velocities (``Lattice.move_particles``).

Host orchestration only: every step runs in the library's kernels.
"""
from __future__ import annotations


class Coupled:
    def __init__(self, lat, dem):
        assert lat.nsph == dem.n, "the lattice and the particle state must hold the same spheres"
        self.lat, self.dem = lat, dem

    def step(self, n: int = 1):
        """n coupled steps; the sphere state stays in device memory (the
        forces, the particle state and the remap's input are CUDA tensors)"""
        for _ in range(int(n)):
            self.lat.step(1)
            hydro = self.lat.particle_forces_device()
            self.dem.step(hydro)
            c, v, w = self.dem.state_device()
            self.lat.move_particles_device(c, v, w)

    def step_host(self, n: int = 1):
        """the same through host arrays (fsl_move_particles)"""
        for _ in range(int(n)):
            self.lat.step(1)
            hydro = self.lat.particle_forces()
            self.dem.step(hydro)
            c, v, w = self.dem.state()
            self.lat.move_particles(c, v, w)
