"""MI355X-native multivariate DTW nearest-neighbour search (TC-DTW, arXiv 2101.07731)."""
