"""Writes heat1d_sigma.txt: the singular values of the implicit-Euler
transfer operator T = M^{-m} of the 1D heat equation (n = 255 interior
points, h = 1/256, dt = 1/1024, m = 64).  T is symmetric with the discrete
sine vectors as eigenvectors, so its singular values are
(1 + dt*4/h^2*sin^2(j*pi*h/2))^{-m}, j = 1..15, the discrete counterpart of
the exponential decay sigma_{R+1} = exp(-(R+1)^2 pi^2 dT) quoted for the
exact solution operator in Sec. 4.1 (Experiment 1).  Closed form only; no
oracle or library code is used."""
import math
import os

h, dt, m = 1.0 / 256, 1.0 / 1024, 64
vals = [(1 + dt * 4 / h ** 2 * math.sin(j * math.pi * h / 2) ** 2) ** (-m) for j in range(1, 16)]
with open(os.path.join(os.path.dirname(os.path.abspath(__file__)), "heat1d_sigma.txt"), "w") as fh:
    fh.write("# sigma_j, j=1..15, of T = (I + dt A)^{-64}, 1D heat, n=255, dt=1/1024 (closed form)\n")
    for v in vals:
        fh.write("%.17e\n" % v)
