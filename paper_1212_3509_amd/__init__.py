"""MI355X (gfx950) library for the separable sinc-quadrature stray-field
operator of arXiv 1212.3509.  The Python side only marshals arguments to the
HIP library (see api.py); inputs.py generates seeded synthetic inputs."""
