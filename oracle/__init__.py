"""FP64 CPU oracle for the batched projective-dynamics membrane step.

TEST INFRASTRUCTURE ONLY. Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import this package. The GPU library
(``paper_2011_04332_amd``) never imports, links or calls it, and it never
imports the library: the two share no code. The only common inputs come from
``npfem_workload`` (seeded geometry and forces, no solver arithmetic).

What it computes, and where that comes from:

* The solid is governed by the elastodynamics equation (eq. 2: rho0 phi'' =
  div P + rho0 b), discretised as a mass-lumped linear finite-element membrane
  (Introduction).
* The time integrator is projective dynamics: the solver derives from ShapeOp
  / projective dynamics (Implementation and architecture). Each implicit step
  minimises (m/2h^2)|q - s|^2 + sum_i (w_i/2) dist^2(S_i q, C_i) by alternating
  exact per-element projections (local step) with one constant SPD linear
  solve (global step).
* The body energy is a sum of weighted elemental potentials (section "Setting
  up new materials"); here: per-triangle strain and area, per-hinge bending,
  per-cell volume.

The paper prints no discretised formulas; every formula here is the published
projective-dynamics method instantiated for these four potentials; where the
paper leaves a choice open, the function that makes it says which reading it
takes.

Modules: ``operators`` (rest-shape operators and the system matrix),
``projections`` (local step), ``solver`` (step / rollout / energy), ``newton``
(brute-force minimiser used to pin convergence), ``gradients`` (finite
differences of rollouts).
"""
