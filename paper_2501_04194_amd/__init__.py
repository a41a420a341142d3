"""STL robustness on MI355X (gfx950): the masking approach of arXiv 2501.04194."""
