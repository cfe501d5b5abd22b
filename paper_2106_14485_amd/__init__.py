"""MI355X-native graph-structured multi-marginal Sinkhorn for dynamic multi-commodity flow."""
