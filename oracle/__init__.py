"""CPU oracle for the hybrid volume-surface integral equation (VSIE) operator.

TEST INFRASTRUCTURE ONLY. Only the test suite, the smoke check and the benchmark's CPU-baseline
leg may import this package. The GPU library never calls it and shares no code with it.

Plain, slow FP64 NumPy: every block of the coupled system (paper Sec. III, eq. (11)) is
assembled densely by direct quadrature and applied by an O(N^2) product. Two operators exist:

  * ``O_direct``: the fully assembled coupled system of eq. (11) (the paper's "method I");
  * ``O_same``  : the compressed hybrid operator of eq. (15) written out densely -- the volume
    block is the same dense Galerkin matrix (the FFT path must reproduce it exactly), the near
    conductor/body block is the precorrected-FFT operator W^T T W + corrections (eq. (13)),
    the far coupling is the tensor train of eq. (14) reconstructed from given cores, and the
    near-far conductor block is the low-rank product U V^* of eq. (12) from given factors.

Conventions (readings of the paper, listed with reasons in the design notes):
  * time dependence exp(+i w t); scalar Green function g = exp(-i k0 R) / (4 pi R) with a single
    1/(4 pi) (eq. (3) prints the factor twice);
  * complex susceptibility chi = eps_r - 1 - i sigma / (w eps0) (eq. (1) writes only eps_r - 1);
  * every row of the coupled system is multiplied by i w eps0 and body rows are tested with the
    field (eq. (4) divided by chi), which makes the matrix complex symmetric as in eq. (8);
  * air voxels (chi = 0) carry identity rows and columns;
  * PWC basis, q = 3, unknown order [j_far | j_near | j_body^x | j_body^y | j_body^z] with
    voxels i1 fastest.

Parity status per function is stated in each module header.
"""
