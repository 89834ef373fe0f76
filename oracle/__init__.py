"""FP64 CPU oracle for the generalized Poisson / Poisson-Boltzmann PCG solver.

TEST INFRASTRUCTURE ONLY.  This package is a plain, slow, obviously correct
restatement of the method of Fisicaro et al., "A generalized Poisson and
Poisson-Boltzmann solver for electrostatic environments" (J. Chem. Phys. 144,
014103 (2016); arXiv:1509.00680).  Only the test suite, the smoke check and the
CPU-baseline leg of the benchmark may import it.  The product library (the HIP
path behind include/gps.h) never calls it, and it shares no code with that
library: every formula here is written out again from the paper.

Modules
  green    -- vacuum Poisson solver G_bc for free / surface / periodic boundary
              conditions (Sec. II.C: the SPe solver used as preconditioner),
              plus dense O(N^2) versions for tiny grids.
  stencil  -- order-2M central second differences and the fixed correction
              vector q = sqrt(eps) lap sqrt(eps) (Sec. II.B, Eq. corr).
  pcg      -- Algorithm PCG with the preconditioner of Eq. PCGdef and the
              operator identity of Eq. corr / Eq. corrPB.
  pb       -- ionic charge (Eqs. ionsconcPB, ionsconcMPB, maxconc) and the
              self-consistent loops of Algorithms SCPB and SCPBimproved.
  dense    -- dense direct solve of the same discrete problem (tiny grids).
  sc       -- Algorithm SC and the PSD minimization (Sec. II.A), with their
              dense operator for tiny grids.
  wire     -- the wire-BC kernel (periodic z, isolated x and y): cell-averaged
              2 K0(|kz| rho) per z mode (Sec. II.C lists the wire BC).
  cavity   -- rigid cavity of Eq. RigCav with its analytic q (Sec. IV.A), and
              the polarization charge of Eqs. rhoiter / remap / rhopol with
              order-2M first differences.

Every floating-point quantity is IEEE binary64.  Grid fields are numpy arrays
of shape (nz, ny, nx), x fastest, cell-centred: point (i, j, k) sits at
((i - (nx-1)/2) h, (j - (ny-1)/2) h, (k - (nz-1)/2) h).

Parity status: every function is pinned by tests/test_oracle_*.py against
closed forms, brute force or limits, except where a docstring says
"parity unpinned".
"""

BC_FREE = "free"
BC_SURFACE = "surface"      # periodic in x and y, free in z
BC_WIRE = "wire"            # periodic in z, free in x and y
BC_PERIODIC = "periodic"
BCS = (BC_FREE, BC_SURFACE, BC_PERIODIC, BC_WIRE)
