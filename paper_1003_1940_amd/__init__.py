"""MI355X-native bi-directed de Bruijn graph construction (k-mer node table and
canonical bi-directed edge list) by sorting, after Kundeti et al."""
