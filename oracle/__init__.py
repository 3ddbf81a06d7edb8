"""FP64 CPU oracle of the hybrid thermal pseudopotential LB boiling model.

TEST INFRASTRUCTURE ONLY.  The oracle is the slow, obviously correct reference
that the GPU library is checked against.  Only ``tests/``, the smoke check in
``__graft_entry__`` and the CPU-baseline leg of ``bench.py`` may import it; the
product package never does, and it shares no code with the GPU library.

Every function is a thin ctypes wrapper over ``lbb_oracle.c`` (and the adjoint
in ``lbb_oracle_adjoint.c``); the arithmetic lives in the C sources, where each
routine cites the equation of the paper (arXiv:1501.03857) that it follows.
"""
from .oracle import (  # noqa: F401
    OracleError,
    Params,
    State,
    COUPLED,
    ISOTHERMAL,
    THERMAL_ONLY,
    lib,
    num_threads,
    Tc,
    kappa,
    phi,
    dphi_dT,
    p_eos,
    dp_dT,
    dp_drho,
    maxwell,
    lattice,
    feq,
    forcing_moments,
    collide_site,
    interaction_force,
    thermal_rhs,
    grad_iso,
    lattice3,
    feq3,
    collide_site3,
    grad_iso3,
    State3,
)
