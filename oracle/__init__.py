"""Plain FP64 CPU oracle of the Galilean PIC step (GEM-PIC, arXiv 2509.16793).

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import or run anything in this
package.  The product path (the HIP library and its Python binding) never
routes through it, and the two share no code: this package imports neither
the binding nor anything compiled, and it holds its own unit conversion, its
own counter-based generator, its own FFT usage and its own linear solves.

Every step is written for a reader to check against the paper by eye:

* ``params``   -- normalisation (Sec. 3, normalised Maxwell units) and the
                  slow-step bound (Sec. 4.2, CFL-like condition).
* ``rng``      -- SplitMix64 counter generator (Steele, Lea & Flood, 2014).
* ``plasma``   -- macro-particle weights (Sec. 5.1, beam/initialised weight Q_b),
                  stratified loading and moving-window injection.
* ``push``     -- CIC gather; relativistic push along the characteristics of
                  the transformed Vlasov equation (Sec. 5, d zeta/d eta = v_z - 1)
                  with the Higuera-Cary rotation.
* ``deposit``  -- charge-conserving (Esirkepov) deposition on the zeta grid and
                  the lab current j = W + rho e_z (Sec. 5.1, current of beam
                  particles j = q n v).
* ``fields``   -- the semi-implicit FD-spectral scheme of Sec. 4.1 solved node
                  by node as a direct 6x6 complex linear system per transverse
                  mode, marched right to left; transverse FFT (Sec. 3.1).
* ``sim``      -- the step in order, the stable tile sort and FP64 diagnostics.
* ``conv3d``   -- plain conv3d forward/backward for the learned denoiser.

Readings where the paper is silent, garbled or inconsistent are named where
they are used (e.g. "reading: ...").
"""
