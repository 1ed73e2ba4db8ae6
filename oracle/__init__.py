"""FP64 CPU oracle of the VR-NeRF renderer hot path -- TEST INFRASTRUCTURE ONLY.

A plain, slow, obviously-correct NumPy renderer written from the paper
(VR-NeRF, arXiv 2311.02542).  It exists to check the HIP renderer and to
time a CPU baseline; only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import it.  The product path never
calls it, and it imports nothing from the product package: it consumes the
plain field/camera dicts drawn by the seeded generators.

Modules (each function cites the passage it follows):
  pq         Sec. 4.1, Eq. 1-2: PQ encode / decode.
  rays       Sec. 4.2.1: canonical FP32 rays and the FP64 cone pitch.
  march      Sec. 4.3: dense-masked lattice march over the occupancy bitfield,
             plus an independent FP64 Amanatides-Woo traversal used as a pin.
  encoding   Sec. 4 (iNGP hash grid), Sec. 4.2.1 Eq. 3 and App. D: hash
             encoding with LOD weights and skipped fine levels.
  sh         real spherical harmonics of the view direction.
  mlp        Sec. 6 (density MLP 1x64, color MLP 2x64, sigmoid in PQ units).
  composite  front-to-back alpha compositing with early termination.
  render     the whole per-pixel pipeline.
  field_io   the oracle's own reader of field files.

Parity status: every stage is pinned by a closed form, invariant, brute
force or library special case in tests/test_oracle_*.py; the whole-image
result has no printed value in the paper ("parity unpinned" at image level,
pinned stage by stage).
"""
