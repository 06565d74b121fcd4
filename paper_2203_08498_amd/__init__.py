"""MI355X (gfx950) implementation of error-vector-sampling accelerated ICCG.

Iwashita, Ikehara, Fukaya, Mifune: "Convergence Acceleration of Preconditioned
CG Solver Based on Error Vector Sampling for a Sequence of Linear Systems"
(arXiv 2203.08498).  The solver is the HIP library ``libesd.so`` behind the C
ABI of ``include/esd.h``; ``esd`` is its ctypes binding and ``autograd`` the
torch.autograd.Function built on it.  ``problems`` generates the synthetic
workloads.
"""
