"""MI355X (gfx950) query path of hybrid spectral-temporal diffusion."""
