"""MI355X-native length-bucketed word sort (arXiv:1411.5283's method on gfx950)."""
